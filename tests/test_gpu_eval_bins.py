"""Large point queries through the C ABI: from 2^16 points on, the points of
a model whose gathers would miss the caches are sorted by bin (16 slabs
per axis) and, where a slab's control points fit in LDS, evaluated bin by
bin from LDS; otherwise by gathers in bin order.  Either way every point's
value, gradient and second derivatives must be the bits of the same point
queried directly (below 2^16 points, no ordering), for scattered points,
points outside the box, on slab boundaries, on knots, on the box faces and
crowded into one bin; the FP64 oracle checks a sample."""

from __future__ import annotations

import numpy as np
import pytest

from gpu_helpers import BF16_REL, F16_REL, FP32_REL, normwise, torch_mod
from helpers import oracle_model
from oracle import bspline as ob
from oracle import quant
from paper_2204_11762_amd import workloads as wl

pytestmark = pytest.mark.gpu

SLABS = 16
MAX_LDS = 64 * 1024
CHUNK = 50_000          # below the ordering threshold: direct evaluation


def _span(U, n, p, u):
    """Largest s in [p, n-1] with U[s] <= u (n-1 from U[n] on)."""
    if u >= U[n]:
        return n - 1
    return p + int(np.searchsorted(U[p:n], u, side="right")) - 1


def _table_stride(p):
    return (2 * p - 1 + p * (p + 1) // 2 + 3) & ~3


def binned_lds_bytes(spec):
    """LDS of a binned workgroup for this model, 0 where the model is
    evaluated by gathers (rational, or a slab's box beyond 64 KiB): the rule
    the library applies at upload."""
    if spec.weights is not None:
        return 0
    pmax = max(spec.degree)
    ext, nspan = [], 0
    for k in range(3):
        U, n, p = np.asarray(spec.knots[k]), spec.n[k], spec.degree[k]
        most = 0
        for j in range(SLABS):
            lo = _span(U, n, p, j / SLABS)
            hi = n - 1 if j == SLABS - 1 else _span(U, n, p, (j + 1) / SLABS)
            most = max(most, hi - lo + 1)
        ext.append(most + pmax)
        nspan = max(nspan, most)
    box = ext[0] * ext[1] * ext[2]
    kn = (nspan + 2) & ~1
    lds = 3 * kn * 8 + 3 * nspan * _table_stride(pmax) * 4 + 4 * box
    return lds if box <= MAX_LDS and lds <= MAX_LDS else 0


def order_score(spec, store):
    elem = 4 if store == 0 else 2
    planes = 2 if spec.weights is not None else 1
    nel = spec.ctrl.size
    return np.sqrt(planes * elem * (nel + 16)) * (max(spec.degree) + 1) ** 3


def bin_points(spec, rng, m):
    """m points: 60% uniform over the box grown by 5% per side (some
    outside, clamped), 25% crowded into a ball of radius 0.3% of the box
    (a few bins of many work items), and points with one coordinate on a
    slab boundary, on a knot or on a box face."""
    lo = np.asarray(spec.lo, dtype=np.float64)
    hi = np.asarray(spec.hi, dtype=np.float64)
    ext = hi - lo
    parts = [wl.uniform_points(rng, int(0.6 * m), lo - 0.05 * ext, hi + 0.05 * ext)]
    centre = lo + ext * rng.uniform(0.2, 0.8, 3)
    parts.append(centre + 0.003 * ext * rng.uniform(-1, 1, (int(0.25 * m), 3)))
    rest = m - sum(len(q) for q in parts)
    q = wl.uniform_points(rng, rest, lo, hi)
    kind = rng.integers(0, 3, rest)
    ax = rng.integers(0, 3, rest)
    for i in range(rest):
        k = ax[i]
        if kind[i] == 0:
            q[i, k] = lo[k] + ext[k] * (rng.integers(0, SLABS + 1) / SLABS)
        elif kind[i] == 1:
            kv = np.unique(spec.knots[k])
            q[i, k] = lo[k] + ext[k] * kv[rng.integers(0, len(kv))]
        else:
            q[i, k] = hi[k] if rng.random() < 0.5 else lo[k]
    parts.append(q)
    xyz = np.concatenate(parts)
    return xyz[rng.permutation(len(xyz))]


def _eval(b, ctx, h, x, mode):
    """Value, gradient (mode >= 1) and Hessian (mode 2) of device points x."""
    torch = torch_mod()
    m = x.shape[0]
    v = torch.full((m,), np.nan, dtype=torch.float32, device="cuda")
    g = torch.full((m, 3), np.nan, dtype=torch.float32, device="cuda") if mode >= 1 else None
    hs = torch.full((m, 6), np.nan, dtype=torch.float32, device="cuda") if mode == 2 else None
    if mode == 2:
        b.mfa_eval_hessian(ctx, h, x, v, hs, g)
    else:
        b.mfa_eval_points(ctx, h, x, v, g)
    torch.cuda.synchronize()
    out = [v.cpu().numpy()]
    if g is not None:
        out.append(g.cpu().numpy())
    if hs is not None:
        out.append(hs.cpu().numpy())
    return out


def _check_same_as_direct(b, ctx, h, xyz, modes=(0, 1, 2)):
    torch = torch_mod()
    x = torch.from_numpy(np.ascontiguousarray(xyz)).cuda()
    n = len(xyz)
    res = {}
    for mode in modes:
        whole = _eval(b, ctx, h, x, mode)
        parts = [_eval(b, ctx, h, x[s:s + CHUNK].contiguous(), mode) for s in range(0, n, CHUNK)]
        for k, arr in enumerate(whole):
            assert np.isfinite(arr).all(), f"mode {mode} output {k}: unwritten or non-finite"
            np.testing.assert_array_equal(arr, np.concatenate([p[k] for p in parts]),
                                          err_msg=f"mode {mode} output {k}")
        res[mode] = whole
    return res


def _oracle_sample(spec, xyz, f, g, rng, rel, ref_ctrl=None, m=1500, grad=True):
    """A sample against the oracle: value and gradient against the stored
    (de-quantised) model, or (grad=False) the value's total error against
    the FP64 model."""
    pick = rng.choice(len(xyz), m, replace=False)
    F, G = ob.eval_world(oracle_model(spec, ctrl=ref_ctrl), xyz[pick])
    ev, eg = normwise(f[pick].astype(np.float64), F), normwise(g[pick].astype(np.float64), G)
    print(f"  oracle sample: value rel {ev:.2e} grad rel {eg:.2e}")
    assert ev <= rel
    if grad:
        assert eg <= rel


def _knots_slab_aligned(n, p):
    """Uniform knots with n - p a multiple of 16: slab boundaries on knots."""
    return wl.clamped_uniform_knots(n, p)


def _knots_double(n, p, at):
    """Uniform knots with interior knot `at` repeated (multiplicity 2)."""
    U = wl.clamped_uniform_knots(n, p).copy()
    U[p + at + 1] = U[p + at]
    return U


def _case(name, rng):
    if name == "fp32_beta_p3":
        return wl.random_model(rng, n=(64, 60, 70), degree=(3, 3, 3), beta_knots=True,
                               lo=(-1, 0, 2), hi=(1, 3, 2.5)), 0
    if name == "bf16_uniform_96":
        return wl.random_model(rng, n=(96, 96, 96), degree=(3, 3, 3)), 1
    if name == "f16_beta_mixed_degrees":
        return wl.random_model(rng, n=(80, 70, 90), degree=(2, 4, 1), beta_knots=True), 2
    if name == "bf16_slab_knots_double_knot":
        deg = (3, 2, 1)
        n = (35, 66, 100)
        knots = (_knots_slab_aligned(n[0], deg[0]), _knots_double(n[1], deg[1], 40),
                 wl.clamped_uniform_knots(n[2], deg[2]))
        ctrl = rng.random((n[2], n[1], n[0]))
        return wl.ModelSpec(deg, knots, ctrl, (0.0, -2.0, 1.0), (4.0, 2.0, 1.5)), 1
    raise KeyError(name)


CASES = ["fp32_beta_p3", "bf16_uniform_96", "f16_beta_mixed_degrees",
         "bf16_slab_knots_double_knot"]
REL = {0: FP32_REL, 1: BF16_REL, 2: F16_REL}


@pytest.mark.parametrize("name", CASES)
def test_binned_equals_direct(mfa, name):
    b, ctx = mfa
    rng = np.random.default_rng(CASES.index(name) + 300)
    spec, store = _case(name, rng)
    assert order_score(spec, store) >= 4e4, "the case must be large enough to be ordered"
    lds = binned_lds_bytes(spec)
    assert lds > 0, "the case must take the binned path"
    xyz = bin_points(spec, rng, 140_000)
    h = b.mfa_model_upload(ctx, spec, store)
    try:
        res = _check_same_as_direct(b, ctx, h, xyz)
        print(f"\n  {name}: {len(xyz)} points, LDS {lds} bytes per workgroup")
        deq = {0: quant.dequant_f32, 1: quant.dequant_bf16, 2: quant.dequant_f16}[store]
        f, g = res[1][0], res[1][1]
        _oracle_sample(spec, xyz, f, g, rng, FP32_REL, ref_ctrl=deq(spec.ctrl))
        _oracle_sample(spec, xyz, f, g, rng, REL[store], grad=False)
    finally:
        b.mfa_model_free(ctx, h)


def test_binned_production_model_bf16(mfa):
    """The 256^3 degree-3 model in BF16 (20^3 control points per slab box),
    2^18 points, against direct evaluation and the de-quantised oracle."""
    b, ctx = mfa
    spec = wl.c3().model
    assert binned_lds_bytes(spec) > 0
    rng = np.random.default_rng(311)
    xyz = bin_points(spec, rng, 1 << 18)
    h = b.mfa_model_upload(ctx, spec, 1)
    try:
        res = _check_same_as_direct(b, ctx, h, xyz, modes=(1,))
        _oracle_sample(spec, xyz, res[1][0], res[1][1], rng, FP32_REL,
                       ref_ctrl=quant.dequant_bf16(spec.ctrl))
    finally:
        b.mfa_model_free(ctx, h)


def test_gathers_in_bin_order_rational(mfa):
    """A rational model is not binned: its points are sorted by bin (the
    probe finds them scattered) and gathered in that order."""
    b, ctx = mfa
    rng = np.random.default_rng(321)
    spec = wl.random_model(rng, n=(60, 50, 40), degree=(3, 2, 3), beta_knots=True)
    spec.weights = rng.uniform(0.2, 5.0, spec.ctrl.shape)
    assert order_score(spec, 0) >= 4e4 and binned_lds_bytes(spec) == 0
    xyz = bin_points(spec, rng, 120_000)
    h = b.mfa_model_upload(ctx, spec, 0)
    try:
        res = _check_same_as_direct(b, ctx, h, xyz, modes=(0, 1))
        M = oracle_model(spec)
        pick = rng.choice(len(xyz), 1500, replace=False)
        F, G = ob.eval_world(M, xyz[pick])
        f, g = res[1][0][pick].astype(np.float64), res[1][1][pick].astype(np.float64)
        assert normwise(f, F) <= FP32_REL and normwise(g, G) <= FP32_REL
    finally:
        b.mfa_model_free(ctx, h)


def test_gathers_in_bin_order_large_slabs(mfa):
    """Knots crowded into the middle of each axis put about 90 spans into
    two slabs: their boxes exceed the LDS, so the model is evaluated by
    gathers in bin order."""
    b, ctx = mfa
    rng = np.random.default_rng(331)
    n, p = 100, 3
    inner = np.sort(rng.uniform(0.44, 0.56, n - p - 1))
    U = np.concatenate([np.zeros(p + 1), inner, np.ones(p + 1)])
    spec = wl.ModelSpec((p, p, p), (U, U.copy(), U.copy()), rng.random((n, n, n)))
    assert order_score(spec, 1) >= 4e4 and binned_lds_bytes(spec) == 0
    xyz = bin_points(spec, rng, 100_000)
    h = b.mfa_model_upload(ctx, spec, 1)
    try:
        res = _check_same_as_direct(b, ctx, h, xyz, modes=(1, 2))
        _oracle_sample(spec, xyz, res[1][0], res[1][1], rng, FP32_REL,
                       ref_ctrl=quant.dequant_bf16(spec.ctrl))
    finally:
        b.mfa_model_free(ctx, h)


def test_single_bin_many_items(mfa):
    """Every point in one bin (more than 20 work items of one bin) and a
    sorted input (already in bin order): both as direct."""
    b, ctx = mfa
    rng = np.random.default_rng(341)
    spec = wl.random_model(rng, n=(96, 96, 96), degree=(3, 3, 3))
    lo = np.array([0.50, 0.25, 0.75]) + 0.001
    xyz = lo + rng.uniform(0.0, 1.0 / SLABS - 0.002, (90_001, 3))
    h = b.mfa_model_upload(ctx, spec, 0)
    try:
        _check_same_as_direct(b, ctx, h, xyz, modes=(1,))
        both = np.concatenate([xyz, bin_points(spec, rng, 60_000)])
        _check_same_as_direct(b, ctx, h, both[wl.morton_order(both)], modes=(0, 2))
    finally:
        b.mfa_model_free(ctx, h)
