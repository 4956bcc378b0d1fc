"""The C ABI library loads without a GPU, exports every entry point that
include/dmpc.h declares, and its host-side checks return the documented codes.
No compute call is made here."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def D():
    import paper_2605_29155_amd as D
    from paper_2605_29155_amd import build
    build.build(force=False)
    return D


def declared_functions():
    text = open(os.path.join(ROOT, "include", "dmpc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dmpc_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dmpc_forward", "dmpc_backward", "dmpc_workspace_bytes", "dmpc_validate", "dmpc_create"):
        assert n in names


def test_every_declared_symbol_is_exported(D):
    L = D.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_validate_codes(D):
    mk = D.make_config
    assert D.validate(mk(4096, 20, flags=D.NEED_GRAD)) == 0
    assert D.validate(mk(0, 1)) == 0
    assert D.validate(mk(-1, 10)) == -1
    assert D.validate(mk(4, 0)) == -1
    assert D.validate(mk(4, 10, max_iter=-1)) == -1
    assert D.validate(mk(4, 2000)) == -2
    assert D.validate(mk(4, 10, max_iter=256)) == -2
    assert D.validate(mk(4, 10, cost_kind=7)) == -2
    assert D.validate(mk(4, 10, flags=0x100)) == -1
    assert D.validate(mk(4, 10, tol_du=float("nan"))) == -1


def test_workspace_bytes(D):
    a = D.workspace_bytes(D.make_config(4096, 20))
    b = D.workspace_bytes(D.make_config(4096, 20, flags=D.NEED_GRAD))
    c = D.workspace_bytes(D.make_config(4096, 20, flags=D.NEED_GRAD | D.PLAIN))
    assert 0 < a < b < c
    assert D.workspace_bytes(D.make_config(4, 2000)) == 0
    # grows linearly in B
    assert D.workspace_bytes(D.make_config(8192, 20)) > 1.9 * a


def test_calls_without_handle_fail_cleanly(D):
    L = D.lib()
    cfg = D.make_config(8, 10)
    p = D.QuadParams(0.75, 2.5e-3, 2.5e-3, 4.5e-3, 0.15, 0.01, 0.05, 9.81)
    rc = L.dmpc_forward(None, C.byref(cfg), p, *([None] * 10), None, 0, None, None)
    assert rc == -1
    assert L.dmpc_mpc_step(None, C.byref(cfg), p, None, None, None, None, None, None) == -1
    rc = L.dmpc_backward(None, C.byref(cfg), D.QuadParams(), None, None, None, None, None, 0, None, None, None, None,
                         None, None, None)
    assert rc == -1
    assert L.dmpc_last_launch_count(None) == -1
    assert b"handle" in L.dmpc_last_error(None)


def test_create_without_gpu_reports_hip_error(D):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    assert D.lib().dmpc_create(C.byref(h), 0) == -3


def test_binding_rejects_host_and_strided_tensors(D):
    import torch
    with pytest.raises(D.DMPCError):
        D._ptr(torch.zeros(4, 13))
    assert D._ptr(None) is None


def test_checkpoint_workspace(D):
    full = D.workspace_bytes(D.make_config(16384, 50, D.COST_DENSE, flags=D.NEED_GRAD))
    ck = D.workspace_bytes(D.make_config(16384, 50, D.COST_DENSE, flags=D.NEED_GRAD, ckpt_every=10))
    assert D.validate(D.make_config(16384, 50, D.COST_DENSE, flags=D.NEED_GRAD, ckpt_every=10)) == 0
    assert D.validate(D.make_config(4, 10, ckpt_every=-1)) == -1
    # stage factors: 1424 bytes per stage; checkpoints: 10 stages of factors + 4 x 1584 bytes
    assert full - ck >= 16384 * (50 - 10) * 1424 - 16384 * 4 * 1584


def test_tuner_entry_points_host_checks(D):
    cfg = D.make_config(64, 20, flags=D.TUNED)
    assert D.validate(cfg) == 0
    c = D.LaunchChoice(0, 1, 1, 0, 0.0)
    L = D.lib()
    assert L.dmpc_set_tuned(None, C.byref(cfg), 1, C.byref(c)) == -1
    assert L.dmpc_get_tuned(None, C.byref(cfg), 1, C.byref(c)) == -1
    assert L.dmpc_last_launch_choice(None, C.byref(c)) == -1
    rc = L.dmpc_autotune(None, C.byref(cfg), D.QuadParams(), None, None, None, None, None, None, None, None, None,
                         None, None, 0, None, None)
    assert rc == -1


def test_tuned_workspace_holds_the_per_launch_buffer(D):
    # a tuned launch may pick the per-launch form, whose linearisation buffer
    # (B x T x 272 floats) must then be part of the workspace
    plain = D.workspace_bytes(D.make_config(256, 20, flags=D.NEED_GRAD | D.PLAIN))
    tuned = D.workspace_bytes(D.make_config(256, 20, flags=D.NEED_GRAD | D.TUNED))
    pers = D.workspace_bytes(D.make_config(256, 20, flags=D.NEED_GRAD))
    assert tuned == plain and tuned - pers >= 256 * 20 * 272 * 4


def test_time_parallel_workspace(D):
    """DMPC_TPAR adds the linearisation buffer, two element buffers of 536
    doubles per instance-stage and one pattern byte per instance-stage."""
    base = D.workspace_bytes(D.make_config(64, 30))
    plain = D.workspace_bytes(D.make_config(64, 30, flags=D.PLAIN))
    tpar = D.workspace_bytes(D.make_config(64, 30, flags=D.TPAR))
    extra = tpar - plain
    assert plain > base
    assert 2 * 64 * 30 * 536 * 8 + 64 * 30 <= extra <= 2 * 64 * 30 * 536 * 8 + 64 * 30 + 2 * 256
    assert D.validate(D.make_config(4, 10, flags=D.TPAR | D.NEED_GRAD)) == 0
    assert D.validate(D.make_config(4, 10, flags=0x80)) == -1
    assert D.validate(D.make_config(4, 10, flags=D.F64_REDO)) == 0
    assert D.validate(D.make_config(4, 10, flags=D.F64_REDO | D.F64)) == -1
    assert D.validate(D.make_config(4, 10, flags=D.F64_REDO | D.PLAIN)) == -2
    # the FP64 form runs as the persistent launch only
    assert D.validate(D.make_config(4, 10, flags=D.F64)) == 0
    assert D.validate(D.make_config(4, 10, flags=D.F64 | D.TPAR)) == -2
    assert D.validate(D.make_config(4, 10, flags=D.F64 | D.PLAIN)) == -2


def test_fp64_form_workspace(D):
    """DMPC_F64 doubles the trajectory and gain regions of the workspace."""
    for B, T in ((64, 20), (1000, 37)):
        a = D.workspace_bytes(D.make_config(B, T))
        b = D.workspace_bytes(D.make_config(B, T, flags=D.F64))
        traj_gains = B * T * (5 * 20 + 68) * 4
        assert abs((b - a) - traj_gains) <= 2 * 256  # regions are 256-byte aligned
