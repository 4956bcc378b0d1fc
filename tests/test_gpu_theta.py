"""GPU tests of the gradient with respect to the model constants (grad_dyn of
dmpc_backward): against the FP64 oracle with the kernel's decisions replayed,
at the gradient bar of 1e-3 (per instance, normwise relative over the eight
constants), and against gravity's closed form through one RK4 step."""
import numpy as np
import pytest

import oracle as orc
import workloads as W

from gpu_util import handle, oracle_replay, rel, run_gpu

pytestmark = pytest.mark.gpu

G_BAR = 1e-3


def _check(d, g, idx=None):
    o = oracle_replay(d, g, idx=idx)
    sel = slice(None) if idx is None else idx
    err = rel(g["gdyn"][sel], o["bwd"]["dtheta"])
    return err, o


@pytest.mark.parametrize("case", ["cfg0", "cfg0_free", "ragged", "dense", "ckpt", "plain", "tpar"])
def test_theta_gradient_matches_oracle(case):
    if case == "cfg0":
        d, kw = W.make(0), {}
    elif case == "cfg0_free":
        d, kw = W.make(0, B=64, T=12, pu_scale=0.01, seed=2101), {}
    elif case == "ragged":
        d, kw = W.make(3, B=64, T=16, seed=2102), {}
        d["T"][:4] = (0, 1, 2, 16)
    elif case == "dense":
        d, kw = W.make(4, B=64, T=12, seed=2103), {}
    elif case == "ckpt":
        d, kw = W.make(0, B=64, T=14, pu_scale=0.01, seed=2104), dict(ckpt=4)
    elif case == "plain":
        d, kw = W.make(0, B=64, T=12, pu_scale=0.01, seed=2105), dict(plain=True)
    else:  # stage factors from the time-parallel tail
        d, kw = W.make(0, B=16, T=20, pu_scale=0.01, seed=2108), dict(tpar=True)
    g = run_gpu(d, theta=True, **kw)
    err, o = _check(d, g)
    assert np.all(np.isfinite(g["gdyn"]))
    assert err.max() <= G_BAR, (case, err.max())
    if case == "ragged":
        assert np.all(g["gdyn"][:2] == 0.0)  # T = 0 and T = 1: no dynamics step


def test_theta_gradient_full_size_sampled():
    d = W.make(1)
    idx = np.arange(0, d["B"], d["B"] // 64)[:64]
    g = run_gpu(d, theta=True)
    err, _ = _check(d, g, idx)
    assert err.max() <= G_BAR, err.max()


def test_theta_path_leaves_the_other_gradients_unchanged():
    d = W.make(0, B=64, T=12, pu_scale=0.01, seed=2106)
    a = run_gpu(d, theta=False)
    b = run_gpu(d, theta=True)
    for k in ("u", "dQ", "dp", "dx0"):
        assert np.array_equal(a[k], b[k]), k


def test_gravity_closed_form_on_the_gpu():
    """Every control held at its upper bound and the upstream gradient on
    v_z and p_z of stage 1 only: dL/dg = -dt - 0.5 dt^2 / 2 exactly (constant
    acceleration through one RK4 step)."""
    B, T = 32, 2
    rng = np.random.default_rng(2107)
    x0 = (W.hover_state(B) + 0.1 * rng.normal(size=(B, 13))).astype(np.float32)
    Q = np.ones((B, T, 17), np.float32)
    p = np.zeros((B, T, 17), np.float32)
    p[..., 13:] = -50.0
    d = dict(x0=x0, Q=Q, p=p, lo=np.zeros((B, 4), np.float32), hi=np.full((B, 4), 3.0, np.float32),
             T=np.full(B, T, np.int32), grad_u=np.zeros((B, T, 4), np.float32), K=10, tol=0.0, T_max=T, B=B,
             cost_kind=0)
    gx = np.zeros((B, T, 13), np.float32)
    gx[:, 1, 9] = 1.0
    gx[:, 1, 2] = 0.5
    g = run_gpu(d, theta=True, grad_x=gx)
    assert np.all(g["u"] == 3.0)
    dt = W.quad_params_f32()["dt"]
    assert np.abs(g["gdyn"][:, 7] - (-dt - 0.25 * dt * dt)).max() <= 1e-6
