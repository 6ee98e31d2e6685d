"""GPU parity of the value and gradient queries (mfa_eval_points) against the
FP64 oracle, through the C ABI."""

import numpy as np
import pytest

from gpu_helpers import BF16_REL, F16_REL, FP32_REL, gpu_eval, normwise
from helpers import oracle_model
from oracle import bspline as ob
from oracle import quant
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _points(spec, rng, m=6000):
    """Random points, every knot plane crossing, box faces/corners, and
    points outside the box (clamped)."""
    lo = np.asarray(spec.lo, dtype=np.float64)
    hi = np.asarray(spec.hi, dtype=np.float64)
    pts = [wl.uniform_points(rng, m, lo, hi)]
    for ax in range(3):
        for kv in np.unique(spec.knots[ax]):
            q = wl.uniform_points(rng, 8, lo, hi)
            q[:, ax] = lo[ax] + kv * (hi[ax] - lo[ax])
            pts.append(q)
    corners = np.array([[a, b, c] for a in (0, 1) for b in (0, 1) for c in (0, 1)], float)
    pts.append(lo + corners * (hi - lo))
    out = wl.uniform_points(rng, 64, lo - 0.5 * (hi - lo), hi + 0.5 * (hi - lo))
    pts.append(out)
    return np.concatenate(pts)


def _check(mfa, spec, store, seed, rel_v, rel_g, ref_ctrl=None):
    b, ctx = mfa
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        rng = np.random.default_rng(seed)
        xyz = _points(spec, rng)
        f, g = gpu_eval(b, ctx, h, xyz)
        M = oracle_model(spec, ctrl=ref_ctrl)
        F, G = ob.eval_world(M, xyz)
        ev, eg = normwise(f, F), normwise(g, G)
        print(f"\n  value rel {ev:.3e}  grad rel {eg:.3e}  (n={len(xyz)})")
        assert np.isfinite(f).all() and np.isfinite(g).all()
        assert ev <= rel_v
        if rel_g is not None:
            assert eg <= rel_g
        # value-only launch gives the same values
        f2, _ = gpu_eval(b, ctx, h, xyz, grad=False)
        np.testing.assert_array_equal(f2, f)
        return ev, eg
    finally:
        b.mfa_model_free(ctx, h)


RANDOM_CASES = [
    # (n, degree, beta knots, lo, hi)
    ((5, 6, 7), (1, 1, 1), False, (0, 0, 0), (1, 1, 1)),
    ((9, 7, 8), (2, 3, 1), True, (-1, 0.5, 2), (1, 1.5, 2.5)),
    ((12, 11, 10), (3, 3, 3), True, (0, 0, 0), (1, 1, 1)),
    ((10, 9, 13), (4, 4, 4), False, (0, 0, 0), (2, 3, 1)),
    ((11, 8, 9), (3, 2, 4), True, (-2, -2, -2), (2, 2, 2)),
    ((5, 4, 3), (4, 3, 2), False, (0, 0, 0), (1, 1, 1)),   # n = p+1: Bezier
]


@pytest.mark.parametrize("case", range(len(RANDOM_CASES)))
@pytest.mark.parametrize("store", [0, 1, 2])
def test_eval_random_models(mfa, case, store):
    n, deg, beta, lo, hi = RANDOM_CASES[case]
    spec = wl.random_model(np.random.default_rng(100 + case), n=n, degree=deg,
                           beta_knots=beta, lo=lo, hi=hi)
    if store == 0:
        _check(mfa, spec, 0, case, FP32_REL, FP32_REL)
    else:
        bound, deq = (BF16_REL, quant.dequant_bf16) if store == 1 else (F16_REL, quant.dequant_f16)
        # against the canonical FP64 model: storage error within the storage bound
        _check(mfa, spec, store, case, bound, None)
        # against the de-quantised model: arithmetic error only, FP32 bound
        _check(mfa, spec, store, case, FP32_REL, FP32_REL, ref_ctrl=deq(spec.ctrl))


def test_eval_c1_model(mfa):
    _check(mfa, wl.c1().model, 0, 1, FP32_REL, FP32_REL)


def test_eval_c2_model(mfa):
    _check(mfa, wl.c2().model, 0, 2, FP32_REL, FP32_REL)


@pytest.fixture(scope="module")
def c3_model():
    return wl.c3().model


def test_eval_c3_model_fp32(mfa, c3_model):
    _check(mfa, c3_model, 0, 3, FP32_REL, FP32_REL)


def test_eval_c3_model_bf16(mfa, c3_model):
    ev, eg = _check(mfa, c3_model, 1, 4, BF16_REL, None)
    _check(mfa, c3_model, 1, 4, FP32_REL, FP32_REL, ref_ctrl=quant.dequant_bf16(c3_model.ctrl))


def test_eval_c3_model_f16(mfa, c3_model):
    _check(mfa, c3_model, 2, 5, F16_REL, None)
    _check(mfa, c3_model, 2, 5, FP32_REL, FP32_REL, ref_ctrl=quant.dequant_f16(c3_model.ctrl))


def _rational_case(seed, degree, n=(7, 8, 6)):
    rng = np.random.default_rng(seed)
    spec = wl.random_model(rng, n=n, degree=degree, beta_knots=True, lo=(-1, 0, 0),
                           hi=(1, 2, 1))
    spec.weights = rng.uniform(0.2, 5.0, spec.ctrl.shape)
    return spec


def _dequant_rational(spec, deq):
    """The stored homogeneous values as a rational model: w*P and w each
    rounded to the storage precision."""
    wq = deq(spec.weights)
    return oracle_model(spec, ctrl=deq(spec.weights * spec.ctrl) / wq), wq


@pytest.mark.parametrize("degree", [(1, 2, 3), (3, 3, 3), (4, 2, 2)])
@pytest.mark.parametrize("store", [0, 1, 2])
def test_eval_rational_models(mfa, degree, store):
    b, ctx = mfa
    spec = _rational_case(200 + sum(degree), degree)
    deq = {0: quant.dequant_f32, 1: quant.dequant_bf16, 2: quant.dequant_f16}[store]
    M, wq = _dequant_rational(spec, deq)
    M.weights = wq
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        xyz = _points(spec, np.random.default_rng(7))
        f, g = gpu_eval(b, ctx, h, xyz)
        F, G = ob.eval_world(M, xyz)
        ev, eg = normwise(f, F), normwise(g, G)
        print(f"\n  rational {degree} store {store}: value rel {ev:.3e}  grad rel {eg:.3e}")
        assert ev <= FP32_REL and eg <= FP32_REL
    finally:
        b.mfa_model_free(ctx, h)


def test_eval_rational_reciprocal_closed_form(mfa):
    """Weights (1, 1, 2) and values (1, 1, 1/2) of degree 2 along x give
    f = 1 / (1 + u^2) exactly (a closed form independent of any evaluator)."""
    b, ctx = mfa
    U2 = np.array([0, 0, 0, 1, 1, 1], float)
    U1 = np.array([0, 0, 1, 1], float)
    ctrl = np.empty((2, 2, 3))
    ctrl[:, :, :] = [1.0, 1.0, 0.5]
    w = np.empty((2, 2, 3))
    w[:, :, :] = [1.0, 1.0, 2.0]
    spec = wl.ModelSpec((2, 1, 1), (U2, U1, U1), ctrl, weights=w)
    h = b.mfa_model_upload(ctx, spec)
    try:
        xyz = wl.uniform_points(np.random.default_rng(3), 4000)
        f, g = gpu_eval(b, ctx, h, xyz)
        u = xyz[:, 0]
        assert normwise(f, 1.0 / (1.0 + u * u)) <= FP32_REL
        gx = -2.0 * u / (1.0 + u * u) ** 2
        assert np.abs(g[:, 0] - gx).max() <= FP32_REL * np.abs(gx).max()
        assert np.abs(g[:, 1:]).max() <= 1e-6
    finally:
        b.mfa_model_free(ctx, h)


def test_eval_zero_points_is_noop(mfa):
    import torch
    b, ctx = mfa
    h = b.mfa_model_upload(ctx, wl.c1().model)
    try:
        x = torch.zeros((0, 3), dtype=torch.float64, device="cuda")
        v = torch.zeros((0,), dtype=torch.float32, device="cuda")
        b.mfa_eval_points(ctx, h, x, v, None)
        torch.cuda.synchronize()
    finally:
        b.mfa_model_free(ctx, h)


def _morton_sorted(xyz, bits=10):
    q = np.clip((xyz * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(len(xyz), dtype=np.int64)
    for bit in range(bits):
        for k in range(3):
            code |= ((q[:, k] >> bit) & 1) << (3 * bit + k)
    return xyz[np.argsort(code, kind="stable")]


def test_locality_order_equals_direct(mfa):
    """From 2^16 points on, queries of a model whose gathers miss the
    caches are sorted by bin on the device (no sort when they arrive in bin
    order) and evaluated bin by bin.  Each point's value, gradient and
    second derivatives are those of the same point queried directly, bit
    for bit: scattered points (sorted), points sorted along a Morton curve
    (left in place), and points outside the box; the oracle checks a
    sample."""
    torch = __import__("torch")
    b, ctx = mfa
    rng = np.random.default_rng(77)
    # 1.07 MB of FP32 control points at degree 3: large enough for the
    # ordering (sqrt(bytes) * (p+1)^3 = 6.6e4 >= 4e4)
    spec = wl.random_model(rng, n=(64, 60, 70), degree=(3, 3, 3), beta_knots=True)
    h = b.mfa_model_upload(ctx, spec)
    n, chunk = 200_003, 50_000            # above and below the ordering threshold
    scattered = wl.uniform_points(rng, n, np.full(3, -0.05), np.full(3, 1.05))
    try:
        for name, xyz in (("scattered", scattered), ("morton", _morton_sorted(scattered))):
            f, g = gpu_eval(b, ctx, h, xyz)
            parts = [gpu_eval(b, ctx, h, xyz[s:s + chunk]) for s in range(0, n, chunk)]
            np.testing.assert_array_equal(f, np.concatenate([p[0] for p in parts]), err_msg=name)
            np.testing.assert_array_equal(g, np.concatenate([p[1] for p in parts]), err_msg=name)
            x = torch.from_numpy(np.ascontiguousarray(xyz)).cuda()
            outs = []
            for lo_i, hi_i in ((0, n),) + tuple((s, min(s + chunk, n)) for s in range(0, n, chunk)):
                m = hi_i - lo_i
                v = torch.full((m,), np.nan, dtype=torch.float32, device="cuda")
                hs = torch.full((m, 6), np.nan, dtype=torch.float32, device="cuda")
                b.mfa_eval_hessian(ctx, h, x[lo_i:hi_i].contiguous(), v, hs)
                torch.cuda.synchronize()
                outs.append(hs.cpu().numpy())
            np.testing.assert_array_equal(outs[0], np.concatenate(outs[1:]), err_msg=name)
            pick = rng.choice(n, 2000, replace=False)
            F, G = ob.eval_world(oracle_model(spec), xyz[pick])
            assert normwise(f[pick], F) <= FP32_REL and normwise(g[pick], G) <= FP32_REL
    finally:
        b.mfa_model_free(ctx, h)
