"""Host build of the GPU's sensitivity step for the gradient w.r.t. the model
constants (paper_2605_29155_amd/csrc/dmpc_theta.hpp), checked on the CPU
against central differences of the oracle's FP64 RK4 map:

  xi'  = A xi + df/dtheta_j                  (lane j's dual-number step)
  eta' = A eta + d(F zt)/dtheta_j            (lane 8 + j's hyper-dual step)

with A = df/dx and F zt = df/dz along zt = (xt, ut), all at (x, u).  The
header is FP32, so the bar is 1e-4 of each output's scale."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

import oracle as orc
import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2605_29155_amd", "csrc", "dmpc_theta.hpp")

SHIM = r"""
#include <cmath>
#define __device__
#define __forceinline__ inline
namespace dmpc_dev { constexpr int NX = 13, NU = 4; }
struct dmpc_quad_params { float mass, Jxx, Jyy, Jzz, arm, kappa, dt, g; };
#include "%s"
extern "C" void step_xi(const float* q, int j, const float* x, const float* u, float* xi) {
  const dmpc_quad_params P{q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7]};
  dmpc_theta::propagate_xi(dmpc_theta::make_pn(P, j), x, u, xi);
}
extern "C" void step_eta(const float* q, int j, const float* x, const float* u, const float* xt, const float* ut,
                         float* eta) {
  const dmpc_quad_params P{q[0], q[1], q[2], q[3], q[4], q[5], q[6], q[7]};
  dmpc_theta::propagate_eta(dmpc_theta::make_pn(P, j), x, u, xt, ut, eta);
}
"""


@pytest.fixture(scope="module")
def lib():
    td = tempfile.mkdtemp()
    src = os.path.join(td, "shim.cpp")
    so = os.path.join(td, "libshim.so")
    open(src, "w").write(SHIM % HDR)
    subprocess.run(["g++", "-O1", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off", "-o", so, src], check=True)
    return C.CDLL(so)


def _f(a):
    return np.ascontiguousarray(a, np.float32)


def _p(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def test_sensitivity_steps_match_central_differences(lib):
    q = W.quad_params_f32()
    names = orc.THETA_NAMES
    th = np.array([q[n] for n in names])
    rng = np.random.default_rng(5)
    x = W.hover_state(1)[0] + np.r_[rng.normal(0, 0.5, 3), rng.normal(0, 0.05, 4), rng.normal(0, 1, 6)]
    x, u = _f(x), _f(1.5 + rng.uniform(0, 1, 4))
    xt, ut = _f(rng.normal(size=13)), _f(rng.normal(size=4))
    xi0, eta0 = _f(rng.normal(size=13)), _f(rng.normal(size=13))
    xd, ud = x.astype(np.float64), u.astype(np.float64)

    def f(thv, xx, uu):
        return orc.rk4(orc.params(*thv), xx, uu)

    # steps large enough that the nested differences are not rounding noise
    he = 1e-4
    for j in range(8):
        h = 1e-4 * th[j]
        tp, tm = th.copy(), th.copy()
        tp[j] += h
        tm[j] -= h
        dfdth = (f(tp, xd, ud) - f(tm, xd, ud)) / (2 * h)
        A_xi = (f(th, xd + he * xi0, ud) - f(th, xd - he * xi0, ud)) / (2 * he)
        A_eta = (f(th, xd + he * eta0, ud) - f(th, xd - he * eta0, ud)) / (2 * he)

        def Fzt(thv):
            return (f(thv, xd + he * xt, ud + he * ut) - f(thv, xd - he * xt, ud - he * ut)) / (2 * he)

        dFzt = (Fzt(tp) - Fzt(tm)) / (2 * h)
        ref_xi, ref_eta = A_xi + dfdth, A_eta + dFzt
        qa = _f(th)
        xi, eta = xi0.copy(), eta0.copy()
        lib.step_xi(_p(qa), j, _p(x), _p(u), _p(xi))
        lib.step_eta(_p(qa), j, _p(x), _p(u), _p(xt), _p(ut), _p(eta))
        assert np.abs(xi - ref_xi).max() <= 1e-4 * max(1.0, np.abs(ref_xi).max()), names[j]
        assert np.abs(eta - ref_eta).max() <= 1e-4 * max(1.0, np.abs(ref_eta).max()), names[j]
