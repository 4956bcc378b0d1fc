"""The oracle's pins must be sensitive: each test here plants one plausible
mistake (a dropped term, a wrong sign or index, a transposed operand) in a
copy of the oracle source, builds it, and checks that the pin suite fails.
Everything runs on the CPU; the real oracle is untouched."""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dmpc_oracle.c")
INC = os.path.join(ROOT, "oracle", "dyn_impl.inc")

# (name, file, original text, mutated text)
MUTANTS = [
    ("drop_KtQux_in_V", SRC, "s += K[a * NX + i] * QuuK[a * NX + j] + K[a * NX + i] * Qux[a * NX + j] +",
     "s += K[a * NX + i] * QuuK[a * NX + j] + 0.0 * Qux[a * NX + j] +"),
    ("sign_v_update", SRC, "s += K[a * NX + i] * Quuk[a] + K[a * NX + i] * q[NX + a] + Qux[a * NX + i] * k[a];",
     "s += K[a * NX + i] * Quuk[a] - K[a * NX + i] * q[NX + a] + Qux[a * NX + i] * k[a];"),
    ("jac_b3y_sign", INC, "Fx[8 * 13 + 3] = -s * 2.0 * qx;", "Fx[8 * 13 + 3] = s * 2.0 * qx;"),
    ("rk4_jac_weights", INC, "static const double wgt[4] = {1.0, 2.0, 2.0, 1.0};",
     "static const double wgt[4] = {1.0, 2.0, 1.0, 2.0};"),
    ("transposed_Atv", SRC, "for (l = 0; l < NX; ++l) s += F[l * NZ + i] * v[l];",
     "for (l = 0; l < NX; ++l) s += (i < NX ? F[i * NZ + l] : F[l * NZ + i]) * v[l];"),
    ("feedback_uses_wrong_index", SRC,
     "s += Kg[(size_t)t * NU * NX + i * NX + j] * (X[t * NX + j] - Xn[t * NX + j]);",
     "s += Kg[(size_t)t * NU * NX + i * NX + j] * (X[t * NX + j] - Xn[(t > 0 ? t - 1 : t) * NX + j]);"),
    ("dx0_sign", SRC, "for (i = 0; i < NX; ++i) dx0[i] = -r[nz + i];", "for (i = 0; i < NX; ++i) dx0[i] = r[nz + i];"),
    ("adjoint_forward_drops_B", SRC, "for (j = 0; j < NU; ++j) s += B[t * NX * NU + i * NU + j] * ut[j];",
     "for (j = 0; j < NU; ++j) s += 0.0 * ut[j];"),
    ("tau_y_sign", INC, "SC ty = a * (-u[0] + u[1] + u[2] - u[3]);", "SC ty = a * (u[0] - u[1] + u[2] - u[3]);"),
    ("quat_kinematics_left_mult", INC, "xd[4] = 0.5 * (qw * wx + qy * wz - qz * wy);",
     "xd[4] = 0.5 * (qw * wx - qy * wz + qz * wy);"),
    ("boxqp_dual_sign", SRC, "if (!(g[i] >= -rel * mag)) ok = 0;", "if (!(g[i] <= rel * mag)) ok = 0;"),
    ("packed_grad_no_symmetrisation", SRC, ": zz[i] * zs[j] + zz[j] * zs[i];", ": zz[i] * zs[j];"),
    ("theta_drops_solution_costate_term", SRC, "acc += lt[i] * (cimag(yc[i]) / h) + ls[i] * (cimag(fz) / h);",
     "acc += lt[i] * (cimag(yc[i]) / h);"),
    ("theta_adjoint_costate_sign", SRC, "gt += A[k * NX + i] * lt[k];", "gt -= A[k * NX + i] * lt[k];"),
    ("theta_solution_costate_transposed", SRC, "gs += A[k * NX + i] * ls[k];", "gs += A[i * NX + k] * ls[k];"),
    ("theta_zt_stage_index", SRC, "for (k = 0; k < NX; ++k) fz += Ac[i * NX + k] * zt[t * NZ + k];",
     "for (k = 0; k < NX; ++k) fz += Ac[i * NX + k] * zt[(t + 1) * NZ + k];"),
    # line search (Sec. IV "Forward pass with line-search") and the objective of eq. (3)
    ("alpha_0125", SRC, "{1.0, 0.5, 0.25, 0.1};", "{1.0, 0.5, 0.25, 0.125};"),
    ("stage_cost_drops_half", SRC, "J += 0.5 * z[i] * s + c[i] * z[i];", "J += z[i] * s + c[i] * z[i];"),
    ("cost_drops_last_stage", SRC, "for (t = 0; t < in->T; ++t) J += stage_cost(",
     "for (t = 0; t + 1 < in->T; ++t) J += stage_cost("),
    ("cost_counts_last_stage_twice", SRC,
     "  for (t = 0; t < in->T; ++t) J += stage_cost(in->C + (size_t)t * NZ * NZ, in->c + t * NZ, X + t * NX, U + t * NU);",
     "  for (t = 0; t < in->T; ++t) J += stage_cost(in->C + (size_t)t * NZ * NZ, in->c + t * NZ, X + t * NX, U + t * NU);"
     " if (in->T > 0) J += stage_cost(in->C + (size_t)(in->T - 1) * NZ * NZ, in->c + (in->T - 1) * NZ,"
     " X + (in->T - 1) * NX, U + (in->T - 1) * NU);"),
    # the check of replayed box-QP patterns
    ("replay_check_multiplier_sign", SRC, "const double wrong = (pat[i] == ORC_LOWER) ? -g : g;",
     "const double wrong = (pat[i] == ORC_LOWER) ? g : -g;"),
    ("replay_check_ignores_box", SRC,
     "const double out = d[i] < a[i] ? a[i] - d[i] : (d[i] > b[i] ? d[i] - b[i] : 0.0);", "const double out = 0.0;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,path,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, path, orig, mut):
    with tempfile.TemporaryDirectory() as td:
        for f in ("dmpc_oracle.c", "dmpc_oracle.h", "dyn_impl.inc"):
            text = open(os.path.join(ROOT, "oracle", f)).read()
            if os.path.basename(path) == f:
                assert text.count(orig) == 1, "mutation anchor not found: " + name
                text = text.replace(orig, mut)
            open(os.path.join(td, f), "w").write(text)
        lib = os.path.join(td, "libmut.so")
        subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", lib,
                        os.path.join(td, "dmpc_oracle.c"), "-lm", "-lpthread"], check=True)
        env = dict(os.environ, DMPC_ORACLE_LIB=lib)
        pins = ["tests/test_golden.py", "tests/test_oracle_dynamics.py", "tests/test_oracle_boxqp.py", "tests/test_oracle_lqr.py",
                "tests/test_oracle_grad.py", "tests/test_oracle_theta.py"]
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider"] + pins,
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, "pins did not catch mutant " + name
