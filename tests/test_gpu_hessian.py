"""GPU parity of the second-derivative queries (mfa_eval_hessian) against
the FP64 oracle's Hessian (derivative control points applied twice), through
the C ABI.

The oracle gets the same FP64 parameters the kernel computes,
u = (x - lo) * (1 / (hi - lo)) clamped to [0, 1], so both take the span
decision at a knot on the same number (second derivatives jump across knots
where the model is only C^1)."""

import numpy as np
import pytest

from gpu_helpers import FP32_REL, gpu_eval, normwise, torch_mod
from helpers import oracle_model
from oracle import bspline as ob
from oracle import quant
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu

# Normwise relative error of the six second derivatives.  Each is a sum of
# (p+1)^3 products in which the second-derivative basis weights alternate in
# sign (they sum to zero), so the FP32 rounding of the weights and of the
# partial sums is amplified by the cancellation: measured up to ~1e-5 on
# these models, bounded here by 10x the first-derivative tolerance.
HESS_REL = 10 * FP32_REL


def _points(spec, rng, m=4000):
    lo = np.asarray(spec.lo, dtype=np.float64)
    hi = np.asarray(spec.hi, dtype=np.float64)
    pts = [wl.uniform_points(rng, m, lo, hi)]
    for ax in range(3):
        for kv in np.unique(spec.knots[ax]):
            q = wl.uniform_points(rng, 6, lo, hi)
            q[:, ax] = lo[ax] + kv * (hi[ax] - lo[ax])
            pts.append(q)
    corners = np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], float)
    pts.append(lo + corners * (hi - lo))
    pts.append(wl.uniform_points(rng, 64, lo - 0.5 * (hi - lo), hi + 0.5 * (hi - lo)))
    return np.concatenate(pts)


def gpu_hessian(b, ctx, model, xyz, grad=True):
    torch = torch_mod()
    x = torch.from_numpy(np.ascontiguousarray(xyz, dtype=np.float64)).cuda()
    n = len(xyz)
    v = torch.full((n,), np.nan, dtype=torch.float32, device="cuda")
    h = torch.full((n, 6), np.nan, dtype=torch.float32, device="cuda")
    g = torch.full((n, 3), np.nan, dtype=torch.float32, device="cuda") if grad else None
    b.mfa_eval_hessian(ctx, model, x, v, h, grad=g)
    torch.cuda.synchronize()
    out = (v.cpu().numpy().astype(np.float64), h.cpu().numpy().astype(np.float64))
    return out + ((g.cpu().numpy().astype(np.float64),) if grad else (None,))


def oracle_hessian(M, xyz):
    """Value, world gradient and world Hessian with the kernel's parameters."""
    lo = np.asarray(M.lo, dtype=np.float64)
    ext = np.asarray(M.hi, dtype=np.float64) - lo
    u = np.clip((xyz - lo) * (1.0 / ext), 0.0, 1.0)
    f, g = ob.eval_local(M, u)
    H = ob.hessian_hodograph(M, u)
    scale = np.array([1.0 / (ext[a] * ext[c]) for a, c in ob.HESS_PAIRS])
    return f, g / ext, H * scale


def _check(mfa, spec, store, seed, ref_ctrl=None, xyz=None):
    b, ctx = mfa
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        rng = np.random.default_rng(seed)
        if xyz is None:
            xyz = _points(spec, rng)
        f, H, g = gpu_hessian(b, ctx, h, xyz)
        M = oracle_model(spec, ctrl=ref_ctrl)
        F, G, HR = oracle_hessian(M, xyz)
        ev, eg, eh = normwise(f, F), normwise(g, G), normwise(H, HR)
        print(f"\n  value rel {ev:.3e}  grad rel {eg:.3e}  hessian rel {eh:.3e}  (n={len(xyz)})")
        assert np.isfinite(f).all() and np.isfinite(g).all() and np.isfinite(H).all()
        assert ev <= FP32_REL and eg <= FP32_REL
        assert eh <= HESS_REL
        # the gradient buffer is optional and does not change the rest
        f2, H2, _ = gpu_hessian(b, ctx, h, xyz, grad=False)
        np.testing.assert_array_equal(f2, f)
        np.testing.assert_array_equal(H2, H)
        # value and gradient agree with the first-derivative query
        f3, g3 = gpu_eval(b, ctx, h, xyz)
        assert normwise(f3, f) <= 1e-6 and normwise(g3, g) <= 1e-6
        return eh
    finally:
        b.mfa_model_free(ctx, h)


CASES = [
    # (n, degree, beta knots, lo, hi)
    ((5, 6, 7), (1, 1, 1), False, (0, 0, 0), (1, 1, 1)),
    ((9, 7, 8), (2, 3, 1), True, (-1, 0.5, 2), (1, 1.5, 2.5)),
    ((12, 11, 10), (3, 3, 3), True, (0, 0, 0), (1, 1, 1)),
    ((10, 9, 13), (4, 4, 4), False, (0, 0, 0), (2, 3, 1)),
    ((11, 8, 9), (3, 2, 4), True, (-2, -2, -2), (2, 2, 2)),
    ((5, 4, 3), (4, 3, 2), False, (0, 0, 0), (1, 1, 1)),   # n = p+1: Bezier
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("store", [0, 1, 2])
def test_hessian_random_models(mfa, case, store):
    n, deg, beta, lo, hi = CASES[case]
    spec = wl.random_model(np.random.default_rng(300 + case), n=n, degree=deg,
                           beta_knots=beta, lo=lo, hi=hi)
    deq = {0: None, 1: quant.dequant_bf16, 2: quant.dequant_f16}[store]
    # stored values de-quantised: the arithmetic error alone
    _check(mfa, spec, store, case, ref_ctrl=None if deq is None else deq(spec.ctrl))


def test_hessian_repeated_knots(mfa):
    """An interior knot of multiplicity p - 1 (C^1 there): second derivatives
    jump at the knot and the right-hand span is taken on both sides."""
    rng = np.random.default_rng(311)
    spec = wl.random_model(rng, n=(10, 9, 8), degree=(3, 3, 3), beta_knots=False)
    knots = list(spec.knots)
    for ax in range(3):
        U = np.array(knots[ax])
        U[4:6] = U[4]               # interior knot U_4 with multiplicity 2
        knots[ax] = U
    spec = wl.ModelSpec(spec.degree, tuple(knots), spec.ctrl, spec.lo, spec.hi)
    _check(mfa, spec, 0, 11)


def test_hessian_polynomial_is_exact(mfa):
    """A model reproducing u^2 v w^3 (Marsden control points): the GPU Hessian
    matches the closed form to FP32 rounding."""
    b, ctx = mfa
    rng = np.random.default_rng(312)
    deg = (3, 2, 4)
    n = (9, 8, 10)
    knots = tuple(wl.clamped_beta_knots(n[k], deg[k], rng) for k in range(3))
    cx, cy, cz = (ob.marsden_coeffs(deg[k], knots[k], e) for k, e in enumerate((2, 1, 3)))
    ctrl = cz[:, None, None] * cy[None, :, None] * cx[None, None, :]
    spec = wl.ModelSpec(deg, knots, ctrl)
    h = b.mfa_model_upload(ctx, spec)
    try:
        u = rng.random((2000, 3))
        f, H, _ = gpu_hessian(b, ctx, h, u)
        x, y, z = u.T
        ref = np.stack([2 * y * z ** 3, 0 * x, 6 * x ** 2 * y * z, 2 * x * z ** 3,
                        6 * x * y * z ** 2, 3 * x ** 2 * z ** 2], axis=1)
        err = normwise(H, ref)
        print(f"\n  u^2 v w^3: hessian rel {err:.3e}")
        assert err <= HESS_REL
        np.testing.assert_allclose(f, x ** 2 * y * z ** 3, rtol=0, atol=1e-6)
    finally:
        b.mfa_model_free(ctx, h)


def test_hessian_c3_model_sampled(mfa):
    """The 256^3 degree-3 render model, 2^20 points in one launch; 3000 of
    them checked against the oracle (FP32 storage and BF16 de-quantised)."""
    b, ctx = mfa
    spec = wl.c3().model
    rng = np.random.default_rng(313)
    xyz = wl.uniform_points(rng, 1 << 20, np.asarray(spec.lo), np.asarray(spec.hi))
    for store, deq in ((0, None), (1, quant.dequant_bf16)):
        h = b.mfa_model_upload(ctx, spec, store)
        try:
            f, H, g = gpu_hessian(b, ctx, h, xyz)
            assert np.isfinite(H).all()
            pick = rng.choice(len(xyz), 3000, replace=False)
            M = oracle_model(spec, ctrl=None if deq is None else deq(spec.ctrl))
            F, G, HR = oracle_hessian(M, xyz[pick])
            eh = normwise(H[pick], HR)
            print(f"\n  c3 store {store}: hessian rel {eh:.3e}")
            assert normwise(f[pick], F) <= FP32_REL and normwise(g[pick], G) <= FP32_REL
            assert eh <= HESS_REL
        finally:
            b.mfa_model_free(ctx, h)


def test_hessian_errors(mfa):
    torch = torch_mod()
    b, ctx = mfa
    spec = wl.random_model(np.random.default_rng(314), n=(6, 6, 6), degree=(2, 2, 2))
    h = b.mfa_model_upload(ctx, spec)
    x = torch.zeros((4, 3), dtype=torch.float64, device="cuda")
    v = torch.zeros(4, dtype=torch.float32, device="cuda")
    hs = torch.zeros((4, 6), dtype=torch.float32, device="cuda")
    try:
        st = b.lib.mfa_eval_hessian(ctx, h, 4, x.data_ptr(), v.data_ptr(), None, None, None)
        assert st == b.MFA_ERR_INVALID
        st = b.lib.mfa_eval_hessian(ctx, h, 0, None, None, None, None, None)
        assert st == b.MFA_OK
        st = b.lib.mfa_eval_hessian(ctx, h, -1, x.data_ptr(), v.data_ptr(), None,
                                    hs.data_ptr(), None)
        assert st == b.MFA_ERR_INVALID
        st = b.lib.mfa_eval_hessian(ctx, h + 999, 4, x.data_ptr(), v.data_ptr(), None,
                                    hs.data_ptr(), None)
        assert st == b.MFA_ERR_HANDLE
    finally:
        b.mfa_model_free(ctx, h)
    rspec = wl.random_model(np.random.default_rng(315), n=(6, 6, 6), degree=(2, 2, 2))
    rspec.weights = np.full(rspec.ctrl.shape, 2.0)
    hr = b.mfa_model_upload(ctx, rspec)
    try:
        st = b.lib.mfa_eval_hessian(ctx, hr, 4, x.data_ptr(), v.data_ptr(), None,
                                    hs.data_ptr(), None)
        assert st == b.MFA_ERR_MODEL
        assert "non-rational" in b.last_error()
    finally:
        b.mfa_model_free(ctx, hr)
