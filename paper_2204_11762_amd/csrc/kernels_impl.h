// HIP kernels for gfx950 (CDNA4): MFA value/gradient queries and the fused
// MFA ray caster.
//
// Per sample (Sect. 3.1, Algorithm 1) a lane
//   1. forms the sample position in FP64 and normalises it to [0,1]^3,
//   2. locates the knot span on each axis (exact FP64 comparisons: a
//      bisection for the first sample of a ray, then a walk, since each
//      coordinate is monotone along a ray),
//   3. evaluates the p+1 non-zero B-spline basis functions and their first
//      derivatives per axis (Cox--de Boor triangle, FP32, reciprocals of
//      the knot differences read from a per-span table),
//   4. gathers the (p+1)^3 control-point block as (p+1)^2 rows of p+1
//      consecutive x values (one bounds-checked buffer load per row) and
//      contracts it sum-factorised: x first (value and d/dx weights), then
//      y, then z, giving the value and all three derivatives at once,
//   5. looks up the RGBA transfer function, applies Phong shading from the
//      analytic gradient, composites front to back and stops the ray once
//      the accumulated opacity exceeds the limit.
// The main ray caster (render_brick_kernel) gives each wave a 4x4 pixel
// tile with four lanes per ray and stages the control points of a round of
// samples in LDS; the global-memory caster (render_global_kernel: when the
// knots or transfer function do not fit in LDS, for rational models, and
// for curvature transfer functions) gives each lane one ray of a 16x16
// tile.  In both, neighbouring rays run in one wave, so their gathers share
// cache lines.  Point queries (eval_kernel, eval_hess_kernel) give each
// lane one point; the latter also returns the second derivatives.  Large
// point queries are sorted by bin first (eval_sort_*) and evaluated bin by
// bin from control points staged in LDS (eval_bin_kernel).
//
// Mixed per-axis degrees run in the kernel of the largest degree P: an axis
// of degree q < P uses the window of P+1 control points that starts at its
// first non-zero function, with zero weights in the last P-q positions.
// The control-point buffer is padded with zeros, so every row load of the
// window stays inside the allocation.

#pragma once

#include <hip/hip_runtime.h>

#include "mfa_dev.h"

namespace mfa {
namespace {

constexpr uint32_t kRsrcWord3 = 0x00020000u;  // raw buffer, 32-bit data format (gfx9)

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes,
                                           (int)kRsrcWord3);
}

// Low and high 16-bit element of a dword as FP32: BF16 (STORE 1) is the
// upper half of an FP32 encoding; FP16 (STORE 2) is IEEE binary16.
template <int STORE>
__device__ __forceinline__ float h16_lo(uint32_t w) {
  if constexpr (STORE == 1)
    return __uint_as_float(w << 16);
  else
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w & 0xffffu));
}
template <int STORE>
__device__ __forceinline__ float h16_hi(uint32_t w) {
  if constexpr (STORE == 1)
    return __uint_as_float(w & 0xffff0000u);
  else
    return (float)__builtin_bit_cast(_Float16, (unsigned short)(w >> 16));
}

// Row of P+1 consecutive control points along x, starting at element e >= 0.
template <int P, int STORE>
__device__ __forceinline__ void load_row(__amdgpu_buffer_rsrc_t rs, int e, float (&r)[P + 1]) {
  if constexpr (STORE == 0) {
    const uint32_t off = (uint32_t)e * 4u;
    if constexpr (P == 1) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
      r[0] = __uint_as_float(v[0]);
      r[1] = __uint_as_float(v[1]);
    } else if constexpr (P == 2) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0);
      r[0] = __uint_as_float(v[0]);
      r[1] = __uint_as_float(v[1]);
      r[2] = __uint_as_float(v[2]);
    } else if constexpr (P == 3) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
      r[0] = __uint_as_float(v[0]);
      r[1] = __uint_as_float(v[1]);
      r[2] = __uint_as_float(v[2]);
      r[3] = __uint_as_float(v[3]);
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b128(rs, off, 0, 0);
      const uint32_t w = __builtin_amdgcn_raw_buffer_load_b32(rs, off + 16u, 0, 0);
      r[0] = __uint_as_float(v[0]);
      r[1] = __uint_as_float(v[1]);
      r[2] = __uint_as_float(v[2]);
      r[3] = __uint_as_float(v[3]);
      r[4] = __uint_as_float(w);
    }
  } else {
    // 16-bit storage: read whole aligned dwords and realign by 16 bits for odd e.
    const uint32_t off = (uint32_t)(e >> 1) * 4u;
    const uint32_t sh = (uint32_t)(e & 1) * 16u;
    if constexpr (P == 1) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
      const uint32_t w0 = __builtin_amdgcn_alignbit(v[1], v[0], sh);
      r[0] = h16_lo<STORE>(w0);
      r[1] = h16_hi<STORE>(w0);
    } else if constexpr (P == 2) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b64(rs, off, 0, 0);
      const uint32_t w0 = __builtin_amdgcn_alignbit(v[1], v[0], sh);
      const uint32_t w1 = __builtin_amdgcn_alignbit(v[1], v[1], sh);
      r[0] = h16_lo<STORE>(w0);
      r[1] = h16_hi<STORE>(w0);
      r[2] = h16_lo<STORE>(w1);
    } else if constexpr (P == 3) {
      const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0);
      const uint32_t w0 = __builtin_amdgcn_alignbit(v[1], v[0], sh);
      const uint32_t w1 = __builtin_amdgcn_alignbit(v[2], v[1], sh);
      r[0] = h16_lo<STORE>(w0);
      r[1] = h16_hi<STORE>(w0);
      r[2] = h16_lo<STORE>(w1);
      r[3] = h16_hi<STORE>(w1);
    } else {
      const auto v = __builtin_amdgcn_raw_buffer_load_b96(rs, off, 0, 0);
      const uint32_t w0 = __builtin_amdgcn_alignbit(v[1], v[0], sh);
      const uint32_t w1 = __builtin_amdgcn_alignbit(v[2], v[1], sh);
      const uint32_t w2 = __builtin_amdgcn_alignbit(v[2], v[2], sh);
      r[0] = h16_lo<STORE>(w0);
      r[1] = h16_hi<STORE>(w0);
      r[2] = h16_lo<STORE>(w1);
      r[3] = h16_hi<STORE>(w1);
      r[4] = h16_lo<STORE>(w2);
    }
  }
}

// ---------------------------------------------------------------------------
// knot spans (exact FP64 comparisons)
// ---------------------------------------------------------------------------

// Largest s in [p, n-1] with U[s] <= u (u in [0,1]); u = 1 gives n-1.
__device__ __forceinline__ int span_search(const double* __restrict__ U, int n, int p, double u) {
  if (u >= U[n]) return n - 1;
  int lo = p, hi = n;  // U[lo] <= u < U[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (U[mid] <= u)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Same result, starting from a nearby span s.
__device__ __forceinline__ int span_walk(const double* __restrict__ U, int n, int p, double u,
                                         int s) {
  while (s < n - 1 && U[s + 1] <= u) ++s;
  while (s > p && U[s] > u) --s;
  return s;
}

// ---------------------------------------------------------------------------
// basis functions of one axis
// ---------------------------------------------------------------------------

// Degree-Q basis N[0..Q] = N_{s-Q..s,Q}(u) and parametric derivatives
// dN[0..Q], from d = u - U_s and the span's table row.  The triangle raises
// the degree one step at a time; at the last step the scaled lower-degree
// values tmp_r = N_{s-Q+1+r,Q-1} / (U_{s+r+1} - U_{s+1-Q+r}) give the
// derivative N'_{s-Q+r,Q} = Q (tmp_{r-1} - tmp_r).
template <int Q>
__device__ __forceinline__ void basis_deg(const float* __restrict__ row, float d, float* N,
                                          float* dN) {
  constexpr int S = table_stride(Q);
  float t[S];
  const float4* r4 = reinterpret_cast<const float4*>(row);
#pragma unroll
  for (int i = 0; i < S / 4; ++i) {
    const float4 v = r4[i];
    t[4 * i + 0] = v.x;
    t[4 * i + 1] = v.y;
    t[4 * i + 2] = v.z;
    t[4 * i + 3] = v.w;
  }
  float left[Q + 1], right[Q + 1];
  left[1] = d;
#pragma unroll
  for (int j = 2; j <= Q; ++j) left[j] = d + t[table_dl(Q, j)];
#pragma unroll
  for (int j = 1; j <= Q; ++j) right[j] = t[table_dr(Q, j)] - d;
  float T[Q];
  N[0] = 1.0f;
#pragma unroll
  for (int q = 1; q <= Q; ++q) {
    float saved = 0.0f;
#pragma unroll
    for (int r = 0; r < q; ++r) {
      const float tmp = N[r] * t[table_inv(Q, q, r)];
      N[r] = fmaf(right[r + 1], tmp, saved);
      saved = left[q - r] * tmp;
      if (q == Q) T[r] = tmp;
    }
    N[q] = saved;
  }
  constexpr float fq = (float)Q;
  dN[0] = -fq * T[0];
#pragma unroll
  for (int r = 1; r < Q; ++r) dN[r] = fq * (T[r - 1] - T[r]);
  dN[Q] = fq * T[Q - 1];
}

// Window of P+1 weights for an axis of runtime degree q <= P: entries
// 0..q hold the non-zero functions, the rest are zero.
template <int P>
__device__ __forceinline__ void axis_basis(int q, const float* __restrict__ row, float d,
                                           float (&N)[P + 1], float (&dN)[P + 1]) {
  if (q == P) {
    basis_deg<P>(row, d, N, dN);
    return;
  }
#pragma unroll
  for (int i = 0; i <= P; ++i) {
    N[i] = 0.0f;
    dN[i] = 0.0f;
  }
  if constexpr (P >= 2) {
    if (q == 1) basis_deg<1>(row, d, N, dN);
  }
  if constexpr (P >= 3) {
    if (q == 2) basis_deg<2>(row, d, N, dN);
  }
  if constexpr (P >= 4) {
    if (q == 3) basis_deg<3>(row, d, N, dN);
  }
}

// Degree-Q basis with first and second parametric derivatives.  The values
// and first derivatives are those of basis_deg.  The second derivatives
// apply the derivative formula twice: the step to degree Q-1 leaves
// tmp1_r = N_{s-Q+2+r,Q-2} / (U_{s+r+1} - U_{s+2-Q+r}), so the degree Q-1
// functions have derivatives D_r = (Q-1)(tmp1_{r-1} - tmp1_r), and
// N''_{s-Q+r,Q} = Q (E_{r-1} - E_r) with E_r = D_r / (U_{s+r+1} - U_{s+1-Q+r}),
// the reciprocal of the last step (entries outside the ranges are 0).  All
// reciprocals come from the span's table row.
template <int Q>
__device__ __forceinline__ void basis_deg2(const float* __restrict__ row, float d, float* N,
                                           float* dN, float* ddN) {
  constexpr int S = table_stride(Q);
  float t[S];
  const float4* r4 = reinterpret_cast<const float4*>(row);
#pragma unroll
  for (int i = 0; i < S / 4; ++i) {
    const float4 v = r4[i];
    t[4 * i + 0] = v.x;
    t[4 * i + 1] = v.y;
    t[4 * i + 2] = v.z;
    t[4 * i + 3] = v.w;
  }
  float left[Q + 1], right[Q + 1];
  left[1] = d;
#pragma unroll
  for (int j = 2; j <= Q; ++j) left[j] = d + t[table_dl(Q, j)];
#pragma unroll
  for (int j = 1; j <= Q; ++j) right[j] = t[table_dr(Q, j)] - d;
  float T[Q], T1[Q];
#pragma unroll
  for (int r = 0; r < Q; ++r) T1[r] = 0.0f;
  N[0] = 1.0f;
#pragma unroll
  for (int q = 1; q <= Q; ++q) {
    float saved = 0.0f;
#pragma unroll
    for (int r = 0; r < q; ++r) {
      const float tmp = N[r] * t[table_inv(Q, q, r)];
      N[r] = fmaf(right[r + 1], tmp, saved);
      saved = left[q - r] * tmp;
      if (q == Q) T[r] = tmp;
      if (q == Q - 1) T1[r] = tmp;
    }
    N[q] = saved;
  }
  constexpr float fq = (float)Q;
  dN[0] = -fq * T[0];
#pragma unroll
  for (int r = 1; r < Q; ++r) dN[r] = fq * (T[r - 1] - T[r]);
  dN[Q] = fq * T[Q - 1];
  if constexpr (Q == 1) {
    ddN[0] = 0.0f;
    ddN[1] = 0.0f;
  } else {
    constexpr float fq1 = (float)(Q - 1);
    float E[Q];
#pragma unroll
    for (int r = 0; r < Q; ++r) {
      const float a = r > 0 ? T1[r - 1] : 0.0f;
      const float b = r < Q - 1 ? T1[r] : 0.0f;
      E[r] = fq1 * (a - b) * t[table_inv(Q, Q, r)];
    }
    ddN[0] = -fq * E[0];
#pragma unroll
    for (int r = 1; r < Q; ++r) ddN[r] = fq * (E[r - 1] - E[r]);
    ddN[Q] = fq * E[Q - 1];
  }
}

template <int P>
__device__ __forceinline__ void axis_basis2(int q, const float* __restrict__ row, float d,
                                            float (&N)[P + 1], float (&dN)[P + 1],
                                            float (&ddN)[P + 1]) {
  if (q == P) {
    basis_deg2<P>(row, d, N, dN, ddN);
    return;
  }
#pragma unroll
  for (int i = 0; i <= P; ++i) {
    N[i] = 0.0f;
    dN[i] = 0.0f;
    ddN[i] = 0.0f;
  }
  if constexpr (P >= 2) {
    if (q == 1) basis_deg2<1>(row, d, N, dN, ddN);
  }
  if constexpr (P >= 3) {
    if (q == 2) basis_deg2<2>(row, d, N, dN, ddN);
  }
  if constexpr (P >= 4) {
    if (q == 3) basis_deg2<3>(row, d, N, dN, ddN);
  }
}

// Uniform knots (U_{p+k} = k/m on an interior span, m = n - p): in the
// normalised coordinate t = (u - U_s) m in [0,1) the p+1 non-zero
// functions are the cardinal B-spline pieces and their t-derivatives.
template <int Q>
__device__ __forceinline__ void cardinal(float t, float* N, float* dN) {
  if constexpr (Q == 1) {
    N[0] = 1.0f - t;
    N[1] = t;
    dN[0] = -1.0f;
    dN[1] = 1.0f;
  } else if constexpr (Q == 2) {
    const float s = 1.0f - t;
    N[0] = 0.5f * s * s;
    N[1] = fmaf(t, s, 0.5f);
    N[2] = 0.5f * t * t;
    dN[0] = -s;
    dN[1] = s - t;
    dN[2] = t;
  } else if constexpr (Q == 3) {
    const float t2 = t * t;
    const float s = 1.0f - t;
    const float s2 = s * s;
    N[0] = s2 * s * (1.0f / 6.0f);
    N[1] = fmaf(t2, fmaf(t, 0.5f, -1.0f), 2.0f / 3.0f);
    N[2] = fmaf(t, fmaf(t, fmaf(t, -0.5f, 0.5f), 0.5f), 1.0f / 6.0f);
    N[3] = t2 * t * (1.0f / 6.0f);
    dN[0] = -0.5f * s2;
    dN[1] = t * fmaf(1.5f, t, -2.0f);
    dN[2] = fmaf(t, fmaf(t, -1.5f, 1.0f), 0.5f);
    dN[3] = 0.5f * t2;
  } else {
    // triangle with the uniform knot differences: left[j] = t + j - 1,
    // right[j] = j - t, every order-q difference equal to q
    float left[Q + 1], right[Q + 1], T[Q];
#pragma unroll
    for (int j = 1; j <= Q; ++j) {
      left[j] = t + (float)(j - 1);
      right[j] = (float)j - t;
    }
    N[0] = 1.0f;
#pragma unroll
    for (int q = 1; q <= Q; ++q) {
      float saved = 0.0f;
#pragma unroll
      for (int r = 0; r < q; ++r) {
        const float tmp = N[r] * (1.0f / (float)q);
        N[r] = fmaf(right[r + 1], tmp, saved);
        saved = left[q - r] * tmp;
        if (q == Q) T[r] = tmp;
      }
      N[q] = saved;
    }
    constexpr float fq = (float)Q;
    dN[0] = -fq * T[0];
#pragma unroll
    for (int r = 1; r < Q; ++r) dN[r] = fq * (T[r - 1] - T[r]);
    dN[Q] = fq * T[Q - 1];
  }
}

// Second t-derivatives of the cardinal pieces of degree Q on a cell: the
// second differences of the degree Q-2 pieces M (M_{-1} = M_{Q-1} = 0),
// N''_r = M_r - 2 M_{r-1} + M_{r-2}; (1, -2, 1) at degree 2 and
// (1 - t, 3t - 2, 1 - 3t, t) at degree 3.
template <int Q>
__device__ __forceinline__ void cardinal_dd(float t, float* ddN) {
  if constexpr (Q == 1) {
    ddN[0] = 0.0f;
    ddN[1] = 0.0f;
  } else if constexpr (Q == 2) {
    ddN[0] = 1.0f;
    ddN[1] = -2.0f;
    ddN[2] = 1.0f;
  } else {
    float M[Q - 1], dM[Q - 1];
    cardinal<Q - 2>(t, M, dM);
#pragma unroll
    for (int r = 0; r <= Q; ++r) {
      const float m0 = r <= Q - 2 ? M[r] : 0.0f;
      const float m1 = (r >= 1 && r - 1 <= Q - 2) ? M[r - 1] : 0.0f;
      const float m2 = r >= 2 ? M[r - 2] : 0.0f;
      ddN[r] = fmaf(-2.0f, m1, m0 + m2);
    }
  }
}

template <int P>
__device__ __forceinline__ void cardinal_dd_window(int q, float t, float (&ddN)[P + 1]) {
  if (q == P) {
    cardinal_dd<P>(t, ddN);
    return;
  }
#pragma unroll
  for (int i = 0; i <= P; ++i) ddN[i] = 0.0f;
  if constexpr (P >= 3) {
    if (q == 2) cardinal_dd<2>(t, ddN);
  }
  if constexpr (P >= 4) {
    if (q == 3) cardinal_dd<3>(t, ddN);
  }
}

// The cubic pieces scaled for the render kernel: 6 N and 2 dN/dt.  With
// s = 1 - t the pieces are s^3, 3t^3 - 6t^2 + 4, 3s^3 - 6s^2 + 4 (the
// mirror image of the second) and t^3, and the scaled derivatives -s^2,
// t (3t - 4), 1 + t (2 - 3t) and t^2, so a sample's value and gradient
// come out of the contraction multiplied by 6^3 and 2 * 6^2; the caller
// folds both factors into its transfer-function and gradient constants.
constexpr float kCubicValueScale = 216.0f;
constexpr float kCubicGradScale = 72.0f;

__device__ __forceinline__ void cardinal3_scaled(float t, float* N, float* dN) {
  // keep the subtractions below as subtractions of the products already
  // formed (not re-fused into multiply-adds)
#pragma clang fp contract(off)
  const float t2 = t * t;
  const float s = 1.0f - t;
  const float s2 = s * s;
  N[0] = s2 * s;
  N[1] = fmaf(t2, fmaf(t, 3.0f, -6.0f), 4.0f);
  N[3] = t2 * t;
  // the pieces sum to 6 and their derivatives to 0: the third of each by
  // subtraction (additions issue at twice the rate of multiplies)
  N[2] = ((6.0f - N[0]) - N[1]) - N[3];
  dN[0] = -s2;
  dN[1] = t * fmaf(t, 3.0f, -4.0f);
  dN[2] = (s2 - dN[1]) - t2;
  dN[3] = t2;
}

template <int P>
__device__ __forceinline__ void cardinal_window(int q, float t, float (&N)[P + 1],
                                                float (&dN)[P + 1]) {
  if (q == P) {
    cardinal<P>(t, N, dN);
    return;
  }
#pragma unroll
  for (int i = 0; i <= P; ++i) {
    N[i] = 0.0f;
    dN[i] = 0.0f;
  }
  if constexpr (P >= 2) {
    if (q == 1) cardinal<1>(t, N, dN);
  }
  if constexpr (P >= 3) {
    if (q == 2) cardinal<2>(t, N, dN);
  }
  if constexpr (P >= 4) {
    if (q == 3) cardinal<3>(t, N, dN);
  }
}

// ---------------------------------------------------------------------------
// sum-factorised contraction of the (P+1)^3 block
// ---------------------------------------------------------------------------

// f = sum N^x_a N^y_b N^z_c P_abc and the three derivative sums, x first:
// each row (b,c) is contracted with N^x and dN^x, then y, then z.
// fetch(b, c, row) supplies row[a] = P_{a,b,c} of the window.
template <int P, bool GRAD, class Fetch>
__device__ __forceinline__ void contract(const float (&N)[3][P + 1], const float (&dN)[3][P + 1],
                                         Fetch fetch, float& f, float (&g)[3]) {
  float a0[P + 1][P + 1], a1[P + 1][P + 1];
#pragma unroll
  for (int c = 0; c <= P; ++c) {
#pragma unroll
    for (int b = 0; b <= P; ++b) {
      float row[P + 1];
      fetch(b, c, row);
      float s0 = N[0][0] * row[0];
      float s1 = dN[0][0] * row[0];
#pragma unroll
      for (int a = 1; a <= P; ++a) {
        s0 = fmaf(N[0][a], row[a], s0);
        if (GRAD) s1 = fmaf(dN[0][a], row[a], s1);
      }
      a0[c][b] = s0;
      a1[c][b] = s1;
    }
  }
  float b0[P + 1], bx[P + 1], by[P + 1];
#pragma unroll
  for (int c = 0; c <= P; ++c) {
    float s0 = N[1][0] * a0[c][0];
    float sx = N[1][0] * a1[c][0];
    float sy = dN[1][0] * a0[c][0];
#pragma unroll
    for (int b = 1; b <= P; ++b) {
      s0 = fmaf(N[1][b], a0[c][b], s0);
      if (GRAD) {
        sx = fmaf(N[1][b], a1[c][b], sx);
        sy = fmaf(dN[1][b], a0[c][b], sy);
      }
    }
    b0[c] = s0;
    bx[c] = sx;
    by[c] = sy;
  }
  float v = N[2][0] * b0[0];
  float gx = N[2][0] * bx[0];
  float gy = N[2][0] * by[0];
  float gz = dN[2][0] * b0[0];
#pragma unroll
  for (int c = 1; c <= P; ++c) {
    v = fmaf(N[2][c], b0[c], v);
    if (GRAD) {
      gx = fmaf(N[2][c], bx[c], gx);
      gy = fmaf(N[2][c], by[c], gy);
      gz = fmaf(dN[2][c], b0[c], gz);
    }
  }
  f = v;
  g[0] = gx;
  g[1] = gy;
  g[2] = gz;
}

// Value, gradient and the six second derivatives (uu, vv, ww, uv, uw, vw),
// sum-factorised like contract(): each row is contracted with N, dN and ddN
// along x; then along y the six combinations that keep at most two
// derivative orders in total; then along z.
template <int P, class Fetch>
__device__ __forceinline__ void contract_hess(const float (&N)[3][P + 1],
                                              const float (&dN)[3][P + 1],
                                              const float (&ddN)[3][P + 1], Fetch fetch,
                                              float& f, float (&g)[3], float (&h)[6]) {
  float v = 0.0f, gx = 0.0f, gy = 0.0f, gz = 0.0f;
  float hxx = 0.0f, hyy = 0.0f, hzz = 0.0f, hxy = 0.0f, hxz = 0.0f, hyz = 0.0f;
  // one z slice c at a time, so that only its rows' sums are live
#pragma unroll
  for (int c = 0; c <= P; ++c) {
    // x: row (b, c) contracted with N, dN and ddN
    float a0[P + 1], a1[P + 1], a2[P + 1];
#pragma unroll
    for (int b = 0; b <= P; ++b) {
      float row[P + 1];
      fetch(b, c, row);
      float s0 = N[0][0] * row[0], s1 = dN[0][0] * row[0], s2 = ddN[0][0] * row[0];
#pragma unroll
      for (int i = 1; i <= P; ++i) {
        s0 = fmaf(N[0][i], row[i], s0);
        s1 = fmaf(dN[0][i], row[i], s1);
        s2 = fmaf(ddN[0][i], row[i], s2);
      }
      a0[b] = s0;
      a1[b] = s1;
      a2[b] = s2;
    }
    // y: (x order, y order) = (0,0) (1,0) (0,1) (2,0) (1,1) (0,2)
    float y00 = 0.0f, y10 = 0.0f, y01 = 0.0f, y20 = 0.0f, y11 = 0.0f, y02 = 0.0f;
#pragma unroll
    for (int b = 0; b <= P; ++b) {
      y00 = fmaf(N[1][b], a0[b], y00);
      y10 = fmaf(N[1][b], a1[b], y10);
      y01 = fmaf(dN[1][b], a0[b], y01);
      y20 = fmaf(N[1][b], a2[b], y20);
      y11 = fmaf(dN[1][b], a1[b], y11);
      y02 = fmaf(ddN[1][b], a0[b], y02);
    }
    // z
    v = fmaf(N[2][c], y00, v);
    gx = fmaf(N[2][c], y10, gx);
    gy = fmaf(N[2][c], y01, gy);
    gz = fmaf(dN[2][c], y00, gz);
    hxx = fmaf(N[2][c], y20, hxx);
    hyy = fmaf(N[2][c], y02, hyy);
    hzz = fmaf(ddN[2][c], y00, hzz);
    hxy = fmaf(N[2][c], y11, hxy);
    hxz = fmaf(dN[2][c], y10, hxz);
    hyz = fmaf(dN[2][c], y01, hyz);
  }
  f = v;
  g[0] = gx;
  g[1] = gy;
  g[2] = gz;
  h[0] = hxx;
  h[1] = hyy;
  h[2] = hzz;
  h[3] = hxy;
  h[4] = hxz;
  h[5] = hyz;
}

// ---------------------------------------------------------------------------
// value and gradient query at arbitrary points (global-memory gathers)
// ---------------------------------------------------------------------------

// Knot span of u on axis A, the largest s in [p, n-1] with U[s] <= u (n-1
// from U[n] on).  Uniform knots: walked from the cell of u m, which is the
// span or next to it.
__device__ __forceinline__ int query_span(const AxisDev& A, bool uniform, double u) {
  if (uniform) {
    const int s0 = min(A.p + (int)(u * A.m), A.n - 1);
    return span_walk(A.knots, A.n, A.p, u, s0);
  }
  return span_search(A.knots, A.n, A.p, u);
}

// Whether span s of an axis with uniform knots is interior: the 2q knots
// around it (U_{s-q+1} .. U_{s+q}) are equally spaced, so the cardinal
// pieces give its basis functions.
__device__ __forceinline__ bool uniform_interior(const AxisDev& A, int s) {
  const int q = A.p, c = s - q, m = A.n - q;
  return c >= q - 1 && c <= m - q;
}

// Basis functions and u-derivatives of one axis at u in span s.  Uniform
// knots on an interior span: the cardinal pieces at t = u m - (s - p), the
// derivatives times m; otherwise the triangle with the span's table row at
// d = u - U_s.
template <int P>
__device__ __forceinline__ void query_basis(const AxisDev& A, bool uniform, int s, double u,
                                            double us, const float* row, float (&N)[P + 1],
                                            float (&dN)[P + 1]) {
  if (uniform && uniform_interior(A, s)) {
    const float t = (float)(u * A.m - (double)(s - A.p));
    cardinal_window<P>(A.p, t, N, dN);
    const float mf = (float)A.m;
#pragma unroll
    for (int r = 0; r <= P; ++r) dN[r] *= mf;
  } else {
    axis_basis<P>(A.p, row, (float)(u - us), N, dN);
  }
}

// The same with second u-derivatives (times m^2 on interior spans).
template <int P>
__device__ __forceinline__ void query_basis2(const AxisDev& A, bool uniform, int s, double u,
                                             double us, const float* row, float (&N)[P + 1],
                                             float (&dN)[P + 1], float (&ddN)[P + 1]) {
  if (uniform && uniform_interior(A, s)) {
    const float t = (float)(u * A.m - (double)(s - A.p));
    cardinal_window<P>(A.p, t, N, dN);
    cardinal_dd_window<P>(A.p, t, ddN);
    const float mf = (float)A.m, m2 = mf * mf;
#pragma unroll
    for (int r = 0; r <= P; ++r) {
      dN[r] *= mf;
      ddN[r] *= m2;
    }
  } else {
    axis_basis2<P>(A.p, row, (float)(u - us), N, dN, ddN);
  }
}

// Value f and world-space gradient g at parameters u (each in [0,1]).
// span[] carries the spans between calls along one ray; first = true
// locates them from scratch.  CARD: on uniform knots, spans walked from
// the cell of u m and cardinal pieces on interior spans (the point
// queries); the global-memory caster keeps the bisection and the triangle,
// which it needs fewer scalar registers for.  RAT: rs holds w*P and rsw holds w; the value
// is the quotient of the two contractions and the gradient follows from the
// quotient rule, (grad A - f grad D) / D.
template <int P, int STORE, bool GRAD, bool RAT, bool CARD = true>
__device__ __forceinline__ void query(const ModelDev& m, __amdgpu_buffer_rsrc_t rs,
                                      __amdgpu_buffer_rsrc_t rsw, const double (&u)[3],
                                      int (&span)[3], bool first, float& f, float (&g)[3]) {
  float N[3][P + 1], dN[3][P + 1];
  int w[3];
  const bool uni = CARD && m.uniform != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const AxisDev& A = m.ax[k];
    const int s = first ? query_span(A, uni, u[k])
                        : span_walk(A.knots, A.n, A.p, u[k], span[k]);
    span[k] = s;
    const float* row = A.tab + (size_t)(s - A.p) * (size_t)table_stride(A.p);
    query_basis<P>(A, uni, s, u[k], A.knots[s], row, N[k], dN[k]);
    w[k] = s - A.p;
  }
  const int e0 = w[0] + m.nx * w[1] + m.nxy * w[2];
  const int nx = m.nx, nxy = m.nxy;
  contract<P, GRAD>(
      N, dN,
      [&](int b, int c, float (&row)[P + 1]) { load_row<P, STORE>(rs, e0 + b * nx + c * nxy, row); },
      f, g);
  if constexpr (RAT) {
    float d, gd[3];
    contract<P, GRAD>(
        N, dN,
        [&](int b, int c, float (&row)[P + 1]) {
          load_row<P, STORE>(rsw, e0 + b * nx + c * nxy, row);
        },
        d, gd);
    const float inv = 1.0f / d;
    f *= inv;
    if (GRAD) {
#pragma unroll
      for (int k = 0; k < 3; ++k) g[k] = (g[k] - f * gd[k]) * inv;
    }
  }
  if (GRAD) {
    g[0] *= m.ax[0].gscale;
    g[1] *= m.ax[1].gscale;
    g[2] *= m.ax[2].gscale;
  }
}

// Value f, world gradient g and world Hessian h (xx, yy, zz, xy, xz, yz) at
// parameters u of a non-rational model; span[] as in query().  The
// parametric second derivative d2f/du_k du_l is scaled by the two
// reciprocal box extents.
template <int P, int STORE, bool CARD = true>
__device__ __forceinline__ void query_hess(const ModelDev& m, __amdgpu_buffer_rsrc_t rs,
                                           const double (&u)[3], int (&span)[3], bool first,
                                           float& f, float (&g)[3], float (&h)[6]) {
  float N[3][P + 1], dN[3][P + 1], ddN[3][P + 1];
  int w[3];
  const bool uni = CARD && m.uniform != 0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const AxisDev& A = m.ax[k];
    const int s = first ? query_span(A, uni, u[k])
                        : span_walk(A.knots, A.n, A.p, u[k], span[k]);
    span[k] = s;
    const float* row = A.tab + (size_t)(s - A.p) * (size_t)table_stride(A.p);
    query_basis2<P>(A, uni, s, u[k], A.knots[s], row, N[k], dN[k], ddN[k]);
    w[k] = s - A.p;
  }
  const int e0 = w[0] + m.nx * w[1] + m.nxy * w[2];
  const int nx = m.nx, nxy = m.nxy;
  contract_hess<P>(
      N, dN, ddN,
      [&](int b, int c, float (&row)[P + 1]) { load_row<P, STORE>(rs, e0 + b * nx + c * nxy, row); },
      f, g, h);
  const float sx = m.ax[0].gscale, sy = m.ax[1].gscale, sz = m.ax[2].gscale;
  g[0] *= sx;
  g[1] *= sy;
  g[2] *= sz;
  h[0] *= sx * sx;
  h[1] *= sy * sy;
  h[2] *= sz * sz;
  h[3] *= sx * sy;
  h[4] *= sx * sz;
  h[5] *= sy * sz;
}

// ---------------------------------------------------------------------------
// rays
// ---------------------------------------------------------------------------

struct Ray {
  double o[3];
  double d[3];
  double t0;
  int nr;  // samples on the ray (0 = miss)
};

// Ray through the centre of pixel (r, c) and its samples inside the box.
// Plain FP64 operations in the stated order (no contraction), so that the
// entry parameter and the sample count are the IEEE results of the
// defining formulas.
__device__ __forceinline__ Ray make_ray(const CamParams& a, int r, int c) {
#pragma clang fp contract(off)
  Ray ray;
  const double W = (double)a.width;
  const double H = (double)a.height;
  const double ca = 2.0 * ((double)c + 0.5) / W - 1.0;
  const double cb = 1.0 - 2.0 * ((double)r + 0.5) / H;
  if (a.kind == 0) {
    const double sa = ca * a.cam0;
    const double sb = cb * a.cam1;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ray.o[k] = a.eye[k] + sa * a.R[k] + sb * a.V[k];
      ray.d[k] = a.F[k];
    }
  } else {
    const double sa = ca * a.cam0 * a.cam1;
    const double sb = cb * a.cam0;
    double dv[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) dv[k] = a.F[k] + sa * a.R[k] + sb * a.V[k];
    const double len = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ray.o[k] = a.eye[k];
      ray.d[k] = dv[k] / len;
    }
  }
  double t0 = 0.0, t1 = __builtin_inf();
  bool miss = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double dk = ray.d[k], ok = ray.o[k];
    if (dk != 0.0) {
      const double ta = (a.lo[k] - ok) / dk;
      const double tb = (a.hi[k] - ok) / dk;
      t0 = fmax(t0, fmin(ta, tb));
      t1 = fmin(t1, fmax(ta, tb));
    } else if (ok < a.lo[k] || ok > a.hi[k]) {
      miss = true;
    }
  }
  ray.t0 = t0;
  ray.nr = 0;
  if (!miss && t1 > t0) {
    const double L = floor((t1 - t0) / a.step);
    ray.nr = (int)fmin(L, (double)kMaxSamplesPerRay);
  }
  return ray;
}

// Parameters of sample s: u = clamp((o + t d - lo) / (hi - lo), 0, 1),
// t = t0 + (s + 1/2) step, with the same unfused operations.
__device__ __forceinline__ void sample_params(const CamParams& a, const Ray& ray, int s,
                                              double (&u)[3]) {
#pragma clang fp contract(off)
  const double t = ray.t0 + ((double)s + 0.5) * a.step;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double x = ray.o[k] + t * ray.d[k];
    const double v = (x - a.lo[k]) * a.inv_ext[k];
    u[k] = fmin(fmax(v, 0.0), 1.0);
  }
}

// x^k for a wave-uniform k >= 0 by binary powering: each trailing zero bit
// of k costs one squaring, each further bit one squaring and (if set) one
// multiply into the result.
__device__ __forceinline__ float ipow_uniform(float x, int k) {
  if (k == 0) return 1.0f;
  while ((k & 1) == 0) {
    x *= x;
    k >>= 1;
  }
  float r = x;
  for (k >>= 1; k != 0; k >>= 1) {
    x *= x;
    if (k & 1) r *= x;
  }
  return r;
}

// Per-ray terms of the specular lobe.  With r = 2 (n.l) n - l the
// reflected light direction, r.v = 2 (n.l)(n.v) - l.v, so a ray keeps 2v
// and l.v, and a sample needs only the two dot products g.l and g.(2v).
struct EyeTerms {
  float v2x, v2y, v2z;  // twice the unit direction towards the eye
  float lv;             // l.v
};

__device__ __forceinline__ EyeTerms eye_terms(const RenderArgsDev& a, float vx, float vy,
                                              float vz) {
  EyeTerms t;
  t.v2x = 2.0f * vx;
  t.v2y = 2.0f * vy;
  t.v2z = 2.0f * vz;
  t.lv = a.light[0] * vx + a.light[1] * vy + a.light[2] * vz;
  return t;
}

// Transfer function and Phong shading of a sample of value f and world
// gradient g: shaded colour (sr, sg, sb) and opacity alpha.
// Transfer function of a sample of value f: colour (sr, sg, sb) and alpha.
template <class TfFetch>
__device__ __forceinline__ void tf_sample(const RenderArgsDev& a, float tf_lo, float tf_scale,
                                          float f, TfFetch tf, float& sr, float& sg, float& sb,
                                          float& alpha) {
  float x = (f - tf_lo) * tf_scale;
  x = fminf(fmaxf(x, 0.0f), 1.0f) * (float)(a.ntf - 1);
  const int i = min((int)x, a.ntf - 2);
  const float t = x - (float)i;
  const float4 c0 = tf(i);
  const float4 c1 = tf(i + 1);
  sr = fmaf(t, c1.x - c0.x, c0.x);
  sg = fmaf(t, c1.y - c0.y, c0.y);
  sb = fmaf(t, c1.z - c0.z, c0.z);
  alpha = fmaf(t, c1.w - c0.w, c0.w);
}

// Phong lighting of the colour (sr, sg, sb) with world gradient g.
template <bool SHADE>
__device__ __forceinline__ void phong_sample(const RenderArgsDev& a, const float (&g)[3],
                                             const EyeTerms& eye, float& sr, float& sg,
                                             float& sb) {
  if (SHADE) {
    // n = g / |g|; diffuse |n.l|; specular max(0, r.v)^k
    const float g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
    // 1 / max(|g|, 1e-6)
    const float inv = rsqrtf(fmaxf(g2, 1e-12f));
    const float gl = g[0] * a.light[0] + g[1] * a.light[1] + g[2] * a.light[2];
    const float gv2 = g[0] * eye.v2x + g[1] * eye.v2y + g[2] * eye.v2z;
    const float ndl = gl * inv;
    // r.v of unit vectors is at most 1; the clamps to [0, 1] fold into the
    // producing instructions (the colours are non-negative, so clamping
    // them to [0, 1] is taking min(1, .))
    const float rv = fminf(fmaxf(fmaf(ndl, gv2 * inv, -eye.lv), 0.0f), 1.0f);
    const float spec = a.ks * ipow_uniform(rv, a.shininess);
    const float kdiff = a.ka + a.kd * fabsf(ndl);
    sr = fminf(fmaxf(fmaf(kdiff, sr, spec), 0.0f), 1.0f);
    sg = fminf(fmaxf(fmaf(kdiff, sg, spec), 0.0f), 1.0f);
    sb = fminf(fmaxf(fmaf(kdiff, sb, spec), 0.0f), 1.0f);
  }
}

template <bool SHADE, class TfFetch>
__device__ __forceinline__ void shade_sample(const RenderArgsDev& a, float tf_lo, float tf_scale,
                                             float f, const float (&g)[3], const EyeTerms& eye,
                                             TfFetch tf, float& sr, float& sg, float& sb,
                                             float& alpha) {
  tf_sample(a, tf_lo, tf_scale, f, tf, sr, sg, sb, alpha);
  phong_sample<SHADE>(a, g, eye, sr, sg, sb);
}

// Principal curvatures k1 >= k2 of the isosurface through a point with
// world gradient g and world Hessian h (xx, yy, zz, xy, xz, yz): the two
// tangential eigenvalues of G = P H P / |g|, P = I - n n^T, n = g / |g|.
// T = trace G = (trace H - n.Hn) / |g|; the split |k1 - k2| is
// sqrt(2) times the Frobenius norm of the traceless tangential part
// G - (T/2) P, a sum of squares without cancellation.  0 where
// |g|^2 < 1e-12.
__device__ __forceinline__ void principal_curvatures(const float (&g)[3], const float (&h)[6],
                                                     float& k1, float& k2) {
  const float g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
  if (!(g2 >= 1e-12f)) {
    k1 = 0.0f;
    k2 = 0.0f;
    return;
  }
  const float il = rsqrtf(g2);
  const float n[3] = {g[0] * il, g[1] * il, g[2] * il};
  const float H[3][3] = {{h[0], h[3], h[4]}, {h[3], h[1], h[5]}, {h[4], h[5], h[2]}};
  float Hn[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) Hn[i] = H[i][0] * n[0] + H[i][1] * n[1] + H[i][2] * n[2];
  const float nHn = n[0] * Hn[0] + n[1] * Hn[1] + n[2] * Hn[2];
  const float T = (h[0] + h[1] + h[2] - nHn) * il;
  float S = 0.0f;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = i; j < 3; ++j) {
      const float php = H[i][j] - n[i] * Hn[j] - Hn[i] * n[j] + nHn * n[i] * n[j];
      const float p = (i == j ? 1.0f : 0.0f) - n[i] * n[j];
      const float d = php * il - 0.5f * T * p;
      S += (i == j ? 1.0f : 2.0f) * d * d;
    }
  }
  const float disc = sqrtf(2.0f * S);
  k1 = 0.5f * (T + disc);
  k2 = 0.5f * (T - disc);
}

// Bilinear lookup of the curvature table at (k1, k2), clamped to its range.
__device__ __forceinline__ float4 curvature_lookup(const RenderArgsDev& a, float k1, float k2) {
  const int m = a.ctf_m;
  auto coord = [&](float k, int& i, float& t) {
    const float x = fminf(fmaxf((k - a.ctf_lo) * a.ctf_scale, 0.0f), 1.0f) * (float)(m - 1);
    i = min((int)x, m - 2);
    t = x - (float)i;
  };
  int i1, i2;
  float t1, t2;
  coord(k1, i1, t1);
  coord(k2, i2, t2);
  const float4 c00 = a.ctf[i2 * m + i1], c01 = a.ctf[i2 * m + i1 + 1];
  const float4 c10 = a.ctf[(i2 + 1) * m + i1], c11 = a.ctf[(i2 + 1) * m + i1 + 1];
  float4 lo, hi, o;
  lo.x = fmaf(t1, c01.x - c00.x, c00.x);
  lo.y = fmaf(t1, c01.y - c00.y, c00.y);
  lo.z = fmaf(t1, c01.z - c00.z, c00.z);
  lo.w = fmaf(t1, c01.w - c00.w, c00.w);
  hi.x = fmaf(t1, c11.x - c10.x, c10.x);
  hi.y = fmaf(t1, c11.y - c10.y, c10.y);
  hi.z = fmaf(t1, c11.z - c10.z, c10.z);
  hi.w = fmaf(t1, c11.w - c10.w, c10.w);
  o.x = fmaf(t2, hi.x - lo.x, lo.x);
  o.y = fmaf(t2, hi.y - lo.y, lo.y);
  o.z = fmaf(t2, hi.z - lo.z, lo.z);
  o.w = fmaf(t2, hi.w - lo.w, lo.w);
  return o;
}

// One front-to-back compositing step; false once the accumulated opacity
// exceeds the termination limit.
__device__ __forceinline__ bool composite_one(float ert, float sr, float sg, float sb, float alpha,
                                              float& cr, float& cg, float& cb, float& A) {
  const float wgt = (1.0f - A) * alpha;
  cr = fmaf(wgt, sr, cr);
  cg = fmaf(wgt, sg, cg);
  cb = fmaf(wgt, sb, cb);
  A += wgt;
  return !(A > ert);
}

__device__ __forceinline__ void count_samples(const RenderArgsDev& a, int count, int lane) {
  if (a.samples != nullptr) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) count += __shfl_xor(count, off, 64);
    if (lane == 0 && count != 0) atomicAdd(a.samples, (unsigned long long)count);
  }
}

// ---------------------------------------------------------------------------
// global-memory ray caster: one lane per ray, all data from global memory
// ---------------------------------------------------------------------------

// Used when the knots or transfer function of a request do not fit the LDS
// budget of the brick kernel, for rational models (RAT: the quotient of the
// two contractions) and for curvature transfer functions (CURV: value,
// gradient and Hessian per sample).
template <int P, int STORE, bool SHADE, bool RAT, bool CURV>
__global__ __launch_bounds__(256) void render_global_kernel(RenderArgsDev a) {
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int px = blockIdx.x * 16 + (wave & 1) * 8 + (lane & 7);
  const int py = blockIdx.y * 16 + (wave >> 1) * 8 + (lane >> 3);
  const bool inside = px < a.width && py < a.height;
  int count = 0;
  if (inside) {
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.m.ctrl, a.m.ctrl_bytes);
    const __amdgpu_buffer_rsrc_t rsw = make_rsrc(RAT ? a.m.wctrl : a.m.ctrl,
                                                 RAT ? a.m.wctrl_bytes : a.m.ctrl_bytes);
    const Ray ray = make_ray(a.cam, py, px);
    float cr = 0.0f, cg = 0.0f, cb = 0.0f, A = 0.0f;
    const EyeTerms eye = eye_terms(a, -(float)ray.d[0], -(float)ray.d[1], -(float)ray.d[2]);
    const float4* tfp = a.tf;
    auto tf = [&](int i) { return tfp[i]; };
    int span[3] = {0, 0, 0};
    for (int s = 0; s < ray.nr; ++s) {
      double u[3];
      sample_params(a.cam, ray, s, u);
      float f, g[3];
      float sr, sg, sb, alpha;
      if constexpr (CURV) {
        // curvature transfer function: the curvature table's colour, its
        // opacity times the value table's
        float h[6], k1, k2;
        query_hess<P, STORE, false>(a.m, rs, u, span, s == 0, f, g, h);
        tf_sample(a, a.tf_lo, a.tf_scale, f, tf, sr, sg, sb, alpha);
        principal_curvatures(g, h, k1, k2);
        const float4 cc = curvature_lookup(a, k1, k2);
        sr = cc.x;
        sg = cc.y;
        sb = cc.z;
        alpha *= cc.w;
        phong_sample<SHADE>(a, g, eye, sr, sg, sb);
      } else {
        query<P, STORE, SHADE, RAT, false>(a.m, rs, rsw, u, span, s == 0, f, g);
        shade_sample<SHADE>(a, a.tf_lo, a.tf_scale, f, g, eye, tf, sr, sg, sb, alpha);
      }
      ++count;
      if (!composite_one(a.ert, sr, sg, sb, alpha, cr, cg, cb, A)) break;
    }
    float4 o;
    o.x = cr;
    o.y = cg;
    o.z = cb;
    o.w = A;
    reinterpret_cast<float4*>(a.out)[(size_t)py * (size_t)a.width + (size_t)px] = o;
  }
  count_samples(a, count, lane);
}

// ---------------------------------------------------------------------------
// LDS-brick ray caster
// ---------------------------------------------------------------------------

struct SpanState {
  int s;      // current span
  double lo;  // U_s
  double hi;  // U_{s+1}
};

// Largest s in [p, n-1] with K[s] <= u by bisection (K in LDS).
__device__ __forceinline__ int lds_span_search(const double* K, int n, int p, double u) {
  if (u >= K[n]) return n - 1;
  int lo = p, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (K[mid] <= u)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Move the cached span to the one of u (a few steps at most between
// consecutive samples); knots from LDS.
__device__ __forceinline__ void span_step(const double* K, int n, int p, double u, SpanState& st) {
  if (u >= st.hi && st.s < n - 1) {
    do {
      ++st.s;
      st.lo = st.hi;
      st.hi = K[st.s + 1];
    } while (u >= st.hi && st.s < n - 1);
  } else if (u < st.lo && st.s > p) {
    do {
      --st.s;
      st.hi = st.lo;
      st.lo = K[st.s];
    } while (u < st.lo && st.s > p);
  }
}

// Minimum (MAX = false) or maximum over the 64 lanes of a wave, returned as
// a wave-uniform value.  Butterflies inside each row of 16 lanes by DPP
// (pair swap, quad-half swap, half-row mirror, row mirror), then across
// rows and halves with the row-swapping permutes.  QUAD: v is already the
// same in the four lanes of each aligned quad, so the two in-quad steps
// are skipped.  Every lane of the wave must be active.
template <bool MAX, bool QUAD = false>
__device__ __forceinline__ unsigned wave_reduce_u32(unsigned v) {
  auto op = [](unsigned x, unsigned y) { return MAX ? (x > y ? x : y) : (x < y ? x : y); };
  constexpr int id = MAX ? 0 : -1;
  if constexpr (!QUAD) {
    v = op(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0xB1, 0xF, 0xF, false));
    v = op(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x4E, 0xF, 0xF, false));
  }
  v = op(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x141, 0xF, 0xF, false));
  v = op(v, (unsigned)__builtin_amdgcn_update_dpp(id, (int)v, 0x140, 0xF, 0xF, false));
  const auto r16 = __builtin_amdgcn_permlane16_swap(v, v, false, false);
  v = op(r16[0], r16[1]);
  const auto r32 = __builtin_amdgcn_permlane32_swap(v, v, false, false);
  v = op(r32[0], r32[1]);
  return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Brick z pitch.  A wave's lanes gather rows whose brick offsets differ by
// dx + pitch_y dy + pitch_z dz for small cell offsets (dx, dy, dz); with
// both pitches multiples of four floats, two such rows share an LDS bank
// (of 32) when a dy + c dz = 0 mod 8, where a and c are the pitches in
// groups of four.  pitch_conflicts(a, c) counts the offsets with |dy|,
// |dz| <= 2 that do, the direct neighbours weighted 4; the z pitch is
// raised by the fewest groups of four that reach the least count for a.
constexpr int pitch_conflicts(int a, int c) {
  int n = 0;
  for (int dy = -2; dy <= 2; ++dy)
    for (int dz = -2; dz <= 2; ++dz)
      if ((dy != 0 || dz != 0) && ((a * dy + c * dz) % 8 + 8) % 8 == 0)
        n += (dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) ? 4 : 1;
  return n;
}
// Groups of four to add to a z pitch of residue c for a y pitch of residue
// a (both mod 8).
constexpr int pitch_z_step(int a, int c) {
  int best = pitch_conflicts(a, 0);
  for (int r = 1; r < 8; ++r) best = pitch_conflicts(a, r) < best ? pitch_conflicts(a, r) : best;
  int k = 0;
  while (pitch_conflicts(a, (c + k) % 8) != best) ++k;
  return k;
}
// The steps packed two bits per (a, c), a in [4h, 4h + 4) for half h.
constexpr unsigned long long pitch_z_steps(int h) {
  unsigned long long w = 0;
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 8; ++c)
      w |= (unsigned long long)pitch_z_step(4 * h + a, c) << (2 * (8 * a + c));
  return w;
}
static_assert(pitch_z_step(3, 3) == 1 && pitch_z_step(3, 1) == 0, "pitch table");

// A DPP quad permutation of v.  Every lane's source lies in its own quad,
// so no lane reads an invalid one and the bound control is immaterial; it
// is set so that the compiler folds the move into a consuming VOP2
// instruction (a multiply with a DPP operand instead of a move and a
// multiply).
template <int CTRL>
__device__ __forceinline__ float quad_perm(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Value of lane (group base + q) of each aligned group of L lanes (L = 1, 2
// or 4, so a group never leaves its quad of lanes), by a DPP quad
// permutation.
template <int L, int Q>
__device__ __forceinline__ float group_bcast(float v) {
  if constexpr (L == 1) {
    return v;
  } else {
    constexpr int b0 = (0 & ~(L - 1)) + Q, b1 = (1 & ~(L - 1)) + Q;
    constexpr int b2 = (2 & ~(L - 1)) + Q, b3 = (3 & ~(L - 1)) + Q;
    constexpr int ctrl = b0 | (b1 << 2) | (b2 << 4) | (b3 << 6);
    return quad_perm<ctrl>(v);
  }
}

// Value of the lane D places earlier in each aligned group of L lanes (L = 2
// or 4); a lane with fewer than D predecessors in its group gets the value
// of the group's first lane (callers overwrite it).  DPP quad permutation.
template <int L, int D>
__device__ __forceinline__ float group_prev(float v) {
  static_assert(D >= 1 && D < L, "distance");
  static_assert(L == 2 || L == 4, "group size");
  constexpr int b0 = 0, b1 = 1 >= D ? 1 - D : 0;
  constexpr int b2 = L == 2 ? 2 : (2 >= D ? 2 - D : 0);
  constexpr int b3 = L == 2 ? (3 - D >= 2 ? 3 - D : 2) : (3 >= D ? 3 - D : 0);
  constexpr int ctrl = b0 | (b1 << 2) | (b2 << 4) | (b3 << 6);
  return quad_perm<ctrl>(v);
}

// Value of the previous lane of each aligned group of L lanes (L = 2 or 4),
// the group's first lane taking its last lane's: a rotation by one, DPP
// quad permutation.
template <int L>
__device__ __forceinline__ float group_rotate(float v) {
  static_assert(L == 2 || L == 4, "group size");
  constexpr int ctrl = L == 4 ? (3 | (0 << 2) | (1 << 4) | (2 << 6)) : (1 | (0 << 2) | (3 << 4) | (2 << 6));
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), ctrl, 0xF, 0xF, false));
}

// Sum over each aligned group of L lanes (L = 1, 2 or 4), returned to every
// lane of the group: pair swap, then (L = 4) half-quad swap, by DPP.
template <int L>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (L >= 2)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  if constexpr (L >= 4)
    v += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, false));
  return v;
}

// a / b for 0 <= a < 2^22, b >= 1, with inv_b ~ 1/b: float estimate plus
// one correction step.
__device__ __forceinline__ int div_small(int a, int b, float inv_b) {
  int q = (int)((float)a * inv_b);
  const int r = a - q * b;
  q += (r >= b) ? 1 : 0;
  q -= (r < 0) ? 1 : 0;
  return q;
}

// Ray caster over pixel tiles, one tile per wave.  Workgroup b renders the
// 2x2 tiles of entry b of a list of super-tiles sorted by decreasing
// estimated work, and the hardware starts workgroups in index order, so the
// longest rays start first while the four waves of a workgroup work on
// neighbouring tiles.  LPR lanes share a ray (a tile has 64/LPR rays): lane
// e of a ray evaluates samples e, e+LPR, e+2 LPR, ...; per step of LPR
// samples the lanes form the transmittance in front of each sample by a
// DPP product scan, so all of them agree on the ray's transmittance and on
// where it stops, and each accumulates its own samples' weighted colour
// (the sums are added at the end).
//
// A wave marches its rays in rounds of `spr` samples.  Before a round it
// stages, into its own LDS brick, every control point that the windows of
// its active rays can touch during the round (the box of spans between the
// smallest and largest parameters of the round's first and last samples);
// the round's samples then gather from LDS.  The four waves of a workgroup
// share the transfer function (and knots) in LDS and never wait for each
// other after loading them.  Which wave renders which tile does not change
// any pixel; on the FAST path the round boundaries of a ray (where FP32
// stepping restarts from FP64) depend on the other live rays of its tile,
// which moves results only at rounding level.
//
// Span location.  FAST (uniform knots U_{p+j} = j/m on every axis, every
// degree >= 2): at the start of a round each lane takes, in FP64, the cell
// c = floor(u m) of its first sample and the local coordinate t = u m - c;
// the samples of the round then advance t in FP32 (t + i * dt) and take the
// cell floor(t).  The knots themselves are never read.  A sample within
// rounding of a knot may use the neighbouring polynomial piece, which for
// degree >= 2 gives the same value and gradient up to rounding.  GENERAL:
// every sample's span is located exactly in FP64 against the knots (kept in
// LDS; cached bounds, stepping along the ray).
//
// Round length.  A round starts at `spr` samples and is halved while the
// box of control points it touches exceeds the brick, so that nearly every
// round gathers from LDS; a round that still does not fit at two samples
// per lane gathers from global memory.
template <int P, int STORE, bool SHADE, bool FAST, bool EQ, int LPR, bool CURV = false>
__device__ __forceinline__ void brick_render(const RenderArgsDev& a, int sup) {
  static_assert(LPR == 1 || LPR == 2 || LPR == 4, "lanes per ray");
  constexpr int TW = LPR == 4 ? 4 : 8;        // tile width in pixels
  constexpr int TH = 64 / LPR / TW;           // tile height
  extern __shared__ float4 lds4[];
  char* lds = reinterpret_cast<char*>(lds4);
  const int tid = threadIdx.x;
  const int wave = tid >> 6;
  const int lane = tid & 63;

  // transfer function and knots, shared by the four waves
  float4* tf_lds = lds4;
  for (int i = tid; i < a.ntf; i += 256) tf_lds[i] = a.tf[i];
  double* knots = reinterpret_cast<double*>(lds + a.lds_knots);
  if constexpr (!FAST) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const int nk = a.m.ax[k].n + a.m.ax[k].p + 1;
      for (int i = tid; i < nk; i += 256) knots[a.knot_off[k] + i] = a.m.ax[k].knots[i];
    }
    // the knots are read by the span search of the ray setup below
    __syncthreads();
  }
  float* brick = reinterpret_cast<float*>(lds + a.lds_bricks) + wave * a.brick_cap;
  const double* K[3] = {knots + a.knot_off[0], knots + a.knot_off[1], knots + a.knot_off[2]};
  auto tf = [&](int i) { return tf_lds[i]; };

  const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.m.ctrl, a.m.ctrl_bytes);
  const int ntx = (a.width + TW - 1) / TW;
  const int nx = a.m.nx, nxy = a.m.nxy;
  const int S = a.spr;
  const int ray_lane = lane / LPR;   // ray of this lane within the tile
  const int e = lane % LPR;          // this lane's sample phase
  // world gradient factors: t-derivatives on the FAST path, u-derivatives
  // on the GENERAL path
  float gfac[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    gfac[k] = FAST ? a.m.ax[k].gscale * (float)a.m.ax[k].m : a.m.ax[k].gscale;
  // degree 3 on uniform knots: scaled cubic pieces (value x 216, gradient x 72)
  constexpr bool kScaled = FAST && EQ && P == 3 && !CURV;
  const float tf_lo = kScaled ? a.tf_lo * kCubicValueScale : a.tf_lo;
  const float tf_scale = kScaled ? a.tf_scale * (1.0f / kCubicValueScale) : a.tf_scale;
  if constexpr (kScaled) {
#pragma unroll
    for (int k = 0; k < 3; ++k) gfac[k] *= 1.0f / kCubicGradScale;
  }
  int count = 0;

  // the workgroup renders super-tile sup (2x2 tiles), wave w its quadrant
  const int nsx = (ntx + 1) >> 1;
  const int tx = (sup % nsx) * 2 + (wave & 1);
  const int ty = (sup / nsx) * 2 + (wave >> 1);
  const int px = tx * TW + ray_lane % TW;
  const int py = ty * TH + ray_lane / TW;
  const bool inside = px < a.width && py < a.height;

  // u_k(s) = ua_k + s ub_k: the sample parameters as an affine function of
  // the sample index
  int nr = 0;
  double ua[3] = {0.0, 0.0, 0.0}, ub[3] = {0.0, 0.0, 0.0};
  EyeTerms eye = {0.0f, 0.0f, 0.0f, 0.0f};
  if (inside) {
    const Ray ray = make_ray(a.cam, py, px);
    nr = ray.nr;
    const double t_half = ray.t0 + 0.5 * a.cam.step;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      ua[k] = (ray.o[k] + t_half * ray.d[k] - a.cam.lo[k]) * a.cam.inv_ext[k];
      ub[k] = a.cam.step * ray.d[k] * a.cam.inv_ext[k];
    }
    eye = eye_terms(a, -(float)ray.d[0], -(float)ray.d[1], -(float)ray.d[2]);
  }
  // uniform knots: the transfer function is first read by the samples, so
  // its loads overlap the ray setup above (every wave reaches this barrier)
  if constexpr (FAST) __syncthreads();
  auto param = [&](int s, int k) {
    return fmin(fmax(fma((double)s, ub[k], ua[k]), 0.0), 1.0);
  };

  bool alive = nr > 0;
  // GENERAL: exact span state per axis
  SpanState st[3];
  // FAST: per-lane increment of the local coordinate between the lane's
  // consecutive samples (LPR samples apart)
  float dt[3];
  if constexpr (FAST) {
#pragma unroll
    for (int k = 0; k < 3; ++k) dt[k] = (float)(ub[k] * a.m.ax[k].m * (double)LPR);
  } else {
    if (alive) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double u = param(min(e, nr - 1), k);
        st[k].s = lds_span_search(K[k], a.m.ax[k].n, a.m.ax[k].p, u);
        st[k].lo = K[k][st[k].s];
        st[k].hi = K[k][st[k].s + 1];
      }
    }
  }
  // colour and opacity accumulated by this lane; transmittance of the ray
  float cr = 0.0f, cg = 0.0f, cb = 0.0f, A = 0.0f, T = 1.0f;
  // a sample is composited while the transmittance in front of it is at
  // least this (opacities lie in [0, 1], checked on the host, so T >= 0
  // and ert >= 1 never stops a ray)
  const float t_stop = 1.0f - a.ert;

  for (int s0 = 0, sr = S;; s0 += sr) {
    if (!__any(alive)) break;
    // A round covers samples [s0, s0 + sr) of every live ray of the wave.
    // It starts at the full length and is halved while the control points
    // it touches do not fit the brick, down to two samples per lane.
    int s1, blo[3], bext[3], pitch_y, pitch_z, nel;
    bool fits;
    for (sr = S;; sr >>= 1) {
      s1 = alive ? min(s0 + sr, nr) : s0;
      // spans of the parameter box of the round (with a margin of 1e-6 in
      // u), reduced over the live rays of the wave
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const AxisDev& Ax = a.m.ax[k];
        const int q = EQ ? P : Ax.p;
        unsigned l = 0xFFFFFFFFu, h = 0u;
        if (alive) {
          const double u0 = param(s0, k), u1 = param(s1 - 1, k);
          const double ul = fmax(fmin(u0, u1) - 1e-6, 0.0);
          const double uh = fmin(fmax(u0, u1) + 1e-6, 1.0);
          if constexpr (FAST) {
            // cells of u m; a sample's cell (below) is computed the same way
            const int m = Ax.n - q;
            l = (unsigned)min(max((int)(ul * Ax.m), 0), m - 1);
            h = (unsigned)min(max((int)(uh * Ax.m), 0), m - 1);
          } else {
            // non-negative floats order as their bit patterns
            l = __float_as_uint((float)ul);
            h = __float_as_uint((float)uh);
          }
        }
        // the box of a ray is the same in its LPR lanes
        l = wave_reduce_u32<false, LPR == 4>(l);
        h = wave_reduce_u32<true, LPR == 4>(h);
        int sl, sh;
        if constexpr (FAST) {
          sl = q + (int)l;
          sh = q + (int)h;
        } else {
          sl = lds_span_search(K[k], Ax.n, q, fmin((double)__uint_as_float(l), 1.0));
          sh = lds_span_search(K[k], Ax.n, q, fmin((double)__uint_as_float(h), 1.0));
        }
        blo[k] = uniform_i(sl - q);
        bext[k] = uniform_i(sh - sl + P + 1);
      }
      // x rows padded to whole groups of four; the z pitch raised so that
      // the rows a wave gathers from neighbouring cells spread over the LDS
      // banks (pitch_z_step)
      pitch_y = (bext[0] + 3) & ~3;
      pitch_z = pitch_y * bext[1];
      {
        constexpr unsigned long long lo = pitch_z_steps(0), hi = pitch_z_steps(1);
        const int ra = (pitch_y >> 2) & 7, rc = (pitch_z >> 2) & 7;
        const unsigned long long w = ra < 4 ? lo : hi;
        pitch_z += 4 * (int)((w >> (2 * (8 * (ra & 3) + rc))) & 3ull);
      }
      nel = pitch_z * (bext[2] - 1) + pitch_y * bext[1];
      fits = nel <= a.brick_cap;
      if (fits || sr <= 2 * LPR) break;
    }

    if (fits) {
      // Stage the brick: group gi = ix + gx (jy + bext1 kz) holds the four
      // consecutive x values starting at x = 4 ix of row (jy, kz), at brick
      // offset 4 ix + pitch_y jy + pitch_z kz.  Lane L takes groups L,
      // L + 64, ...; its (ix, jy, kz), global element index and brick
      // offset advance by the mixed-radix digits of 64.
      const int gx = pitch_y >> 2;
      const int gxy = gx * bext[1];
      const int ngroups = gxy * bext[2];
      const float inv_gx = __builtin_amdgcn_rcpf((float)gx);
      const int d_row = uniform_i(div_small(64, gx, inv_gx));
      const int d_ix = 64 - d_row * gx;
      const int d_kz = uniform_i(div_small(d_row, bext[1], __builtin_amdgcn_rcpf((float)bext[1])));
      const int d_jy = d_row - d_kz * bext[1];
      const int dg = 4 * d_ix + nx * d_jy + nxy * d_kz;   // step without carries
      const int dg_c1 = nx - 4 * gx;                      // carry ix -> jy
      const int dg_c2 = nxy - nx * bext[1];               // carry jy -> kz
      // brick offsets: the carry ix -> jy adds pitch_y - 4 gx = 0
      const int dl = 4 * d_ix + pitch_y * d_jy + pitch_z * d_kz;
      const int dl_c2 = pitch_z - pitch_y * bext[1];      // carry jy -> kz
      const int kz = div_small(lane, gxy, __builtin_amdgcn_rcpf((float)gxy));
      const int rem = lane - kz * gxy;
      int jy = div_small(rem, gx, inv_gx);
      int ix = rem - jy * gx;
      int g = (blo[0] + 4 * ix) + nx * (blo[1] + jy) + nxy * (blo[2] + kz);
      int lo = 4 * ix + pitch_y * jy + pitch_z * kz;
      // four groups per lane in flight: loads past the last group read
      // element 0 (and are dropped), only the LDS stores are predicated
      for (int gi = lane; gi < ngroups; gi += 256) {
        float v[4][4];
        int lu[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          load_row<3, STORE>(rs, gi + 64 * u < ngroups ? g : 0, v[u]);
          lu[u] = lo;
          ix += d_ix;
          jy += d_jy;
          g += dg;
          lo += dl;
          if (ix >= gx) {
            ix -= gx;
            jy += 1;
            g += dg_c1;
          }
          if (jy >= bext[1]) {
            jy -= bext[1];
            g += dg_c2;
            lo += dl_c2;
          }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          if (gi + 64 * u < ngroups) {
            float4 w;
            w.x = v[u][0];
            w.y = v[u][1];
            w.z = v[u][2];
            w.w = v[u][3];
            *reinterpret_cast<float4*>(brick + lu[u]) = w;
          }
        }
      }
    }
    const int emax = nel - 1 - (P + P * pitch_y + P * pitch_z);

    // FAST: cell c = floor(u m) (clamped to the spans) and local coordinate
    // u m - c of this lane's first sample of the round, in FP64
    int ca[3] = {0, 0, 0};
    float ta[3] = {0.0f, 0.0f, 0.0f};
    if constexpr (FAST) {
      if (s0 + e < s1) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const AxisDev& Ax = a.m.ax[k];
          const int m = Ax.n - (EQ ? P : Ax.p);
          const double um = param(s0 + e, k) * Ax.m;
          const int c = min(max((int)um, 0), m - 1);
          ca[k] = c;
          ta[k] = (float)(um - (double)c);
        }
      }
    }

    // Interior rounds (uniform knots, every axis of degree P): when every
    // cell of the round's box is interior on all three axes (cardinal
    // pieces apply), so is every sample's cell, since the box holds the
    // cells of all the round's samples with a margin far above the FP32
    // stepping error.  The samples then skip the per-axis range test, and
    // their brick offset is formed in FP32 from the cells' floor values
    // (small integers, exact) on top of a per-lane base.
    constexpr bool kInteriorPath = FAST && EQ && !CURV;
    bool interior = false;
    float basef = 0.0f;
    const float pitch_yf = (float)pitch_y, pitch_zf = (float)pitch_z;
    if constexpr (kInteriorPath) {
      interior = fits;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const int m = a.m.ax[k].n - P;
        // the box's cells are blo .. blo + bext - P - 1
        interior = interior && blo[k] >= P - 1 && blo[k] + bext[k] - P - 1 <= m - P;
      }
      basef = (float)(ca[0] - blo[0]) + pitch_yf * (float)(ca[1] - blo[1]) +
              pitch_zf * (float)(ca[2] - blo[2]);
    }

    // one lane's sample: basis weights and window start of each axis
    auto weights = [&](int s, int i, float (&N)[3][P + 1], float (&dN)[3][P + 1], int (&w)[3]) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const AxisDev& Ax = a.m.ax[k];
        const int q = EQ ? P : Ax.p;
        if constexpr (FAST) {
          const int m = Ax.n - q;
          const float t = fmaf((float)i, dt[k], ta[k]);
          const float fl = floorf(t);
          int c = ca[k] + (int)fl;
          if (c >= q - 1 && c <= m - q) {
            // interior cell: cardinal pieces at the fractional part
            const float tl = t - fl;
            if constexpr (kScaled)
              cardinal3_scaled(tl, N[k], dN[k]);
            else if constexpr (EQ)
              cardinal<P>(tl, N[k], dN[k]);
            else
              cardinal_window<P>(q, tl, N[k], dN[k]);
          } else {
            // boundary span, or a cell that FP32 stepping moved past either
            // end (clamped): triangle with the span's reciprocal table
            c = min(max(c, 0), m - 1);
            const float tl = t - (float)(c - ca[k]);
            const float* row = Ax.tab + (size_t)c * (size_t)table_stride(q);
            axis_basis<P>(q, row, tl * Ax.inv_m, N[k], dN[k]);
            // derivatives to t units, both in the scale of the interior pieces
            const float nsc = kScaled ? 6.0f : 1.0f;
            const float dsc = kScaled ? 2.0f * Ax.inv_m : Ax.inv_m;
#pragma unroll
            for (int r = 0; r <= P; ++r) {
              N[k][r] *= nsc;
              dN[k][r] *= dsc;
            }
          }
          w[k] = c;
        } else {
          const double u = param(s, k);
          span_step(K[k], Ax.n, q, u, st[k]);
          const float d = (float)(u - st[k].lo);
          const float* row = Ax.tab + (size_t)(st[k].s - q) * (size_t)table_stride(q);
          axis_basis<P>(q, row, d, N[k], dN[k]);
          w[k] = st[k].s - q;
        }
      }
    };

    // CURV: basis functions with first and second derivatives of this
    // lane's sample: FAST, in t (cardinal pieces on interior cells, the span
    // table's triangle scaled to t on the boundary spans); GENERAL, in u
    // from the span tables
    auto weights2 = [&](int s, int i, float (&N)[3][P + 1], float (&dN)[3][P + 1],
                        float (&ddN)[3][P + 1], int (&w)[3]) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const AxisDev& Ax = a.m.ax[k];
        const int q = EQ ? P : Ax.p;
        if constexpr (FAST) {
          const int m = Ax.n - q;
          const float t = fmaf((float)i, dt[k], ta[k]);
          const float fl = floorf(t);
          int c = ca[k] + (int)fl;
          if (c >= q - 1 && c <= m - q) {
            const float tl = t - fl;
            if constexpr (EQ) {
              cardinal<P>(tl, N[k], dN[k]);
              cardinal_dd<P>(tl, ddN[k]);
            } else {
              cardinal_window<P>(q, tl, N[k], dN[k]);
              cardinal_dd_window<P>(q, tl, ddN[k]);
            }
          } else {
            c = min(max(c, 0), m - 1);
            const float tl = t - (float)(c - ca[k]);
            const float* row = Ax.tab + (size_t)c * (size_t)table_stride(q);
            axis_basis2<P>(q, row, tl * Ax.inv_m, N[k], dN[k], ddN[k]);
            const float i2 = Ax.inv_m * Ax.inv_m;
#pragma unroll
            for (int r = 0; r <= P; ++r) {
              dN[k][r] *= Ax.inv_m;
              ddN[k][r] *= i2;
            }
          }
          w[k] = c;
        } else {
          const double u = param(s, k);
          span_step(K[k], Ax.n, q, u, st[k]);
          const float d = (float)(u - st[k].lo);
          const int c = st[k].s - q;
          axis_basis2<P>(q, Ax.tab + (size_t)c * (size_t)table_stride(q), d, N[k], dN[k],
                         ddN[k]);
          w[k] = c;
        }
      }
    };
    // CURV: value table, principal curvatures of the isosurface, curvature
    // table (its colour, its opacity times the value table's), then Phong
    auto shade_curv = [&](float f, const float (&g)[3], const float (&h)[6], float& sr,
                          float& sg, float& sb, float& alpha) {
      float gw[3], hw[6];
#pragma unroll
      for (int k = 0; k < 3; ++k) gw[k] = g[k] * gfac[k];
      hw[0] = h[0] * (gfac[0] * gfac[0]);
      hw[1] = h[1] * (gfac[1] * gfac[1]);
      hw[2] = h[2] * (gfac[2] * gfac[2]);
      hw[3] = h[3] * (gfac[0] * gfac[1]);
      hw[4] = h[4] * (gfac[0] * gfac[2]);
      hw[5] = h[5] * (gfac[1] * gfac[2]);
      tf_sample(a, tf_lo, tf_scale, f, tf, sr, sg, sb, alpha);
      float k1, k2;
      principal_curvatures(gw, hw, k1, k2);
      const float4 cc = curvature_lookup(a, k1, k2);
      sr = cc.x;
      sg = cc.y;
      sb = cc.z;
      alpha *= cc.w;
      phong_sample<SHADE>(a, gw, eye, sr, sg, sb);
    };

    // shade(): transfer function and Phong shading of this lane's sample.
    // composite(): front-to-back compositing of the group's samples j, j+1,
    // ..., j+LPR-1 (one per lane); false once the ray terminates.
    // T is the ray's transmittance (1 - accumulated opacity) before the
    // group, the same in its LPR lanes.  The transmittance in front of lane
    // e's sample is T times the product of (1 - alpha) over the group's
    // earlier lanes, an exclusive product scan in two DPP steps.  The
    // sample is composited while that transmittance is at least 1 - ert
    // (the accumulated opacity has not passed ert), with weight
    // transmittance x alpha; each lane accumulates its own weighted colour
    // and weight (opacity), summed over the ray's lanes once at the end.  A
    // sample past the round's end has alpha 0 and changes nothing.
    auto shade = [&](float f, const float (&g)[3], float& sr, float& sg, float& sb,
                     float& alpha) {
      float gw[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) gw[k] = g[k] * gfac[k];
      shade_sample<SHADE>(a, tf_lo, tf_scale, f, gw, eye, tf, sr, sg, sb, alpha);
    };
    auto composite = [&](int j, float sr, float sg, float sb, float alpha, bool valid) {
      const float om = 1.0f - alpha;
      float ex = 1.0f;   // product of (1 - alpha) over the earlier lanes of the group
      if constexpr (LPR >= 2) {
        // lane e takes (1 - alpha) of lane e-1, the first lane 1 (the
        // selection is made on the source: every lane of the group takes
        // part in each DPP move)
        ex = group_rotate<LPR>(e == LPR - 1 ? 1.0f : om);
        if constexpr (LPR == 4) {
          ex *= group_prev<LPR, 1>(ex);   // lanes e-1, e-2
          ex *= group_prev<LPR, 2>(ex);   // and e-3
        }
      }
      const float tb = T * ex;
      const bool reached = tb >= t_stop;
      const float w = reached ? tb * alpha : 0.0f;
      cr = fmaf(w, sr, cr);
      cg = fmaf(w, sg, cg);
      cb = fmaf(w, sb, cb);
      A += w;
      count += (valid && reached) ? 1 : 0;
      T *= group_bcast<LPR, LPR - 1>(ex * om);
      return T >= t_stop;
    };

    // row (b, c) of a sample's window in the brick, e0 its first element
    auto brick_row = [&](int e0) {
      return [=](int b, int c, float (&row)[P + 1]) {
        const float* r = brick + e0 + b * pitch_y + c * pitch_z;
#pragma unroll
        for (int q = 0; q <= P; ++q) row[q] = r[q];
      };
    };

    bool interior_done = false;
    if constexpr (kInteriorPath) {
      if (interior) {
        interior_done = true;
        // local coordinates advance by additions, within the box margin
        float tk[3] = {ta[0], ta[1], ta[2]};
        const float emaxf = (float)emax;
        for (int j = s0; j < s1; j += LPR) {
          // A lane past the round's end evaluates a sample anyway (its
          // window is clamped into the staged brick, so every value is
          // finite) and adds it with alpha 0.
          const bool valid = j + e < s1;
          float sr, sg, sb, alpha, f, g[3];
          float N[3][P + 1], dN[3][P + 1], fl[3];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const float t = tk[k];
            tk[k] = t + dt[k];
            fl[k] = floorf(t);
            const float tl = t - fl[k];
            if constexpr (kScaled)
              cardinal3_scaled(tl, N[k], dN[k]);
            else
              cardinal<P>(tl, N[k], dN[k]);
          }
          const float ef = fmaf(fl[2], pitch_zf, fmaf(fl[1], pitch_yf, fl[0] + basef));
          const int e0 = (int)__builtin_amdgcn_fmed3f(ef, 0.0f, emaxf);
          contract<P, SHADE>(N, dN, brick_row(e0), f, g);
          shade(f, g, sr, sg, sb, alpha);
          alpha = valid ? alpha : 0.0f;
          if (!composite(j, sr, sg, sb, alpha, valid)) {
            alive = false;
            break;
          }
        }
      }
    }

    if (interior_done) {
      // the round was rendered by the interior loop
    } else if (fits) {
      for (int j = s0, i = 0; j < s1; j += LPR, ++i) {
        const int s = j + e;
        // a lane past the round's end adds alpha 0 and colour 0
        float sr = 0.0f, sg = 0.0f, sb = 0.0f, alpha = 0.0f;
        if (s < s1) {
          if constexpr (CURV) {
            float f, g[3], h[6];
            float N[3][P + 1], dN[3][P + 1], ddN[3][P + 1];
            int w[3];
            weights2(s, i, N, dN, ddN, w);
            int e0 = (w[0] - blo[0]) + __mul24(pitch_y, w[1] - blo[1]) +
                     __mul24(pitch_z, w[2] - blo[2]);
            e0 = min(max(e0, 0), emax);
            contract_hess<P>(N, dN, ddN, brick_row(e0), f, g, h);
            shade_curv(f, g, h, sr, sg, sb, alpha);
          } else {
            float f, g[3];
            float N[3][P + 1], dN[3][P + 1];
            int w[3];
            weights(s, i, N, dN, w);
            // 24-bit products: pitches and in-box offsets are far below 2^23
            int e0 = (w[0] - blo[0]) + __mul24(pitch_y, w[1] - blo[1]) +
                     __mul24(pitch_z, w[2] - blo[2]);
            e0 = min(max(e0, 0), emax);
            contract<P, SHADE>(N, dN, brick_row(e0), f, g);
            shade(f, g, sr, sg, sb, alpha);
          }
        }
        if (!composite(j, sr, sg, sb, alpha, s < s1)) {
          alive = false;
          break;
        }
      }
    } else {
      for (int j = s0, i = 0; j < s1; j += LPR, ++i) {
        const int s = j + e;
        // a lane past the round's end adds alpha 0 and colour 0
        float sr = 0.0f, sg = 0.0f, sb = 0.0f, alpha = 0.0f;
        if (s < s1) {
          if constexpr (CURV) {
            float f, g[3], h[6];
            float N[3][P + 1], dN[3][P + 1], ddN[3][P + 1];
            int w[3];
            weights2(s, i, N, dN, ddN, w);
            const int e0 = w[0] + nx * w[1] + nxy * w[2];
            contract_hess<P>(
                N, dN, ddN,
                [&](int b, int c, float (&row)[P + 1]) {
                  load_row<P, STORE>(rs, e0 + b * nx + c * nxy, row);
                },
                f, g, h);
            shade_curv(f, g, h, sr, sg, sb, alpha);
          } else {
            float f, g[3];
            float N[3][P + 1], dN[3][P + 1];
            int w[3];
            weights(s, i, N, dN, w);
            const int e0 = w[0] + nx * w[1] + nxy * w[2];
            contract<P, SHADE>(
                N, dN,
                [&](int b, int c, float (&row)[P + 1]) {
                  load_row<P, STORE>(rs, e0 + b * nx + c * nxy, row);
                },
                f, g);
            shade(f, g, sr, sg, sb, alpha);
          }
        }
        if (!composite(j, sr, sg, sb, alpha, s < s1)) {
          alive = false;
          break;
        }
      }
    }
    if (s1 >= nr) alive = false;
  }
  // the colour and opacity of a ray are the sums of its lanes' parts
  cr = group_sum<LPR>(cr);
  cg = group_sum<LPR>(cg);
  cb = group_sum<LPR>(cb);
  A = group_sum<LPR>(A);
  if (inside && e == 0) {
    float4 o;
    o.x = cr;
    o.y = cg;
    o.z = cb;
    o.w = A;
    reinterpret_cast<float4*>(a.out)[(size_t)py * (size_t)a.width + (size_t)px] = o;
  }
  count_samples(a, count, lane);
}

template <int P, int STORE, bool SHADE, bool FAST, bool EQ, int LPR, bool CURV>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    brick_waves_per_simd(P, FAST, EQ, CURV)))) void render_brick_kernel(RenderArgsDev a) {
  const int sup = uniform_i(a.tile_order[blockIdx.x]);
  if (sup < 0) return;   // empty launch slot of a smaller XCD group
  brick_render<P, STORE, SHADE, FAST, EQ, LPR, CURV>(a, sup);
}

// Request of global super-tile t of a batch class: the largest r with
// base[r] <= t (base holds the prefix sums of the requests' super-tiles).
__device__ __forceinline__ int batch_request(const int32_t* base, int nreq, int t) {
  int lo = 0, hi = nreq;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (base[mid] <= t)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// The same ray caster over the super-tiles of every request of a batch
// class; workgroup b renders entry b of the class's work-sorted list.
template <int P, int STORE, bool SHADE, bool FAST, bool EQ, int LPR>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    brick_waves_per_simd(P, FAST, EQ, false, true)))) void render_batch_kernel(BatchDev b) {
  const int t = uniform_i(b.tile_order[blockIdx.x]);
  const int r = uniform_i(batch_request(b.tile_base, b.nreq, t));
  brick_render<P, STORE, SHADE, FAST, EQ, LPR>(b.args[r], t - b.tile_base[r]);
}

// ---------------------------------------------------------------------------
// tile order: counting sort of the tiles by decreasing estimated work
// ---------------------------------------------------------------------------

constexpr int kBuckets = 512;

// Bucket of a work estimate (8 samples per bucket), largest work first.
__device__ __forceinline__ int cost_rank(int c) { return kBuckets - 1 - min(c >> 3, kBuckets - 1); }

// XCD group of super-tile t of a frame nsx super-tiles wide: square regions
// of region x region super-tiles are dealt to the groups in a skewed
// pattern, so that each group's regions are spread over the image.
__device__ __forceinline__ int xcd_group(int t, int nsx, int region) {
  const int sx = t % nsx, sy = t / nsx;
  return ((sx / region) + 3 * (sy / region)) & (kXcdGroups - 1);
}

// Clear nhist counters: the state in which a frame's planning finds its
// scratch (set up once per buffer, then kept by plan_cost_kernel).
__global__ __launch_bounds__(256) void plan_init_kernel(unsigned* hist, int nhist) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < nhist) hist[i] = 0u;
}

// Work estimate of every super-tile (2x2 tiles of tile_w x tile_h pixels):
// the largest sample count among nine rays (corners, edge midpoints and
// centre of its pixel rectangle).  Part r (0..3) takes rays r, r + 4 and
// r + 8 of the nine (row-major over the 3x3 points).
__device__ __forceinline__ int supertile_cost_part(const RenderArgsDev& a, int t, int r) {
  const int ntx = (a.width + a.tile_w - 1) / a.tile_w;
  const int nsx = (ntx + 1) >> 1;
  const int x0 = (t % nsx) * 2 * a.tile_w, y0 = (t / nsx) * 2 * a.tile_h;
  const int x1 = min(x0 + 2 * a.tile_w - 1, a.width - 1);
  const int y1 = min(y0 + 2 * a.tile_h - 1, a.height - 1);
  int c = 0;
  for (int j = r; j < 9; j += 4) {
    const int jy = j / 3, jx = j - 3 * jy;
    const int y = jy == 0 ? y0 : jy == 1 ? (y0 + y1) >> 1 : y1;
    const int x = jx == 0 ? x0 : jx == 1 ? (x0 + x1) >> 1 : x1;
    c = max(c, make_ray(a.cam, y, x).nr);
  }
  return c;
}

__device__ __forceinline__ int supertile_cost(const RenderArgsDev& a, int t) {
  int c = 0;
  for (int r = 0; r < 4; ++r) c = max(c, supertile_cost_part(a, t, r));
  return c;
}

// Single frame: work estimates and the per-group bucket histogram.  Four
// lanes share a super-tile's nine rays; the histogram is gathered in LDS
// and added to the frame's counters.  Frames on a stream alternate between
// two sets of counters (histogram and cursors); the grid clears the set of
// the previous frame, whose planning is complete, for the next one.
__global__ __launch_bounds__(256) void plan_cost_kernel(RenderArgsDev a) {
  __shared__ unsigned h[kXcdGroups * kBuckets];
  const int tid = threadIdx.x;
  for (int i = blockIdx.x * 256 + tid; i < 2 * kPlanHistWords; i += gridDim.x * 256)
    a.tile_clear[i] = 0u;
  for (int i = tid; i < kXcdGroups * kBuckets; i += 256) h[i] = 0u;
  __syncthreads();
  const int t = blockIdx.x * 64 + (tid >> 2);
  const int r = tid & 3;
  int c = t < a.ntiles ? supertile_cost_part(a, t, r) : 0;
  c = max(c, __shfl_xor(c, 1));
  c = max(c, __shfl_xor(c, 2));
  if (t < a.ntiles && r == 0) {
    a.tile_cost[t] = c;
    atomicAdd(&h[xcd_group(t, a.nsx, a.region) * kBuckets + cost_rank(c)], 1u);
  }
  __syncthreads();
  for (int i = tid; i < kXcdGroups * kBuckets; i += 256)
    if (h[i] != 0u) atomicAdd(&a.tile_hist[i], h[i]);
}

// Exclusive prefix sum of each group's bucket histogram (one workgroup per
// group).
__global__ __launch_bounds__(kBuckets) void plan_scan_kernel(unsigned* hist) {
  __shared__ unsigned v[kBuckets];
  const int tid = threadIdx.x;
  unsigned* h = hist + blockIdx.x * kBuckets;
  const unsigned own = h[tid];
  v[tid] = own;
  __syncthreads();
  for (int off = 1; off < kBuckets; off <<= 1) {
    const unsigned add = tid >= off ? v[tid - off] : 0u;
    __syncthreads();
    v[tid] += add;
    __syncthreads();
  }
  h[tid] = v[tid] - own;
}

// Launch order.  Within its group a super-tile's position follows its
// bucket (every workgroup reserves one range per bucket it holds tiles of,
// so positions are unique; the order within a bucket is arbitrary and
// changes no pixel); slot position * G + group then puts the k-th longest
// super-tile of group g at workgroup index 8 k + g.  G = 1 for batches.
template <int G>
__global__ __launch_bounds__(256) void plan_scatter_kernel(const int* cost, int n, int nsx,
                                                           int region, unsigned* base,
                                                           int* order) {
  __shared__ unsigned cnt[G * kBuckets];
  __shared__ unsigned off[G * kBuckets];
  const int tid = threadIdx.x;
  for (int i = tid; i < G * kBuckets; i += 256) cnt[i] = 0u;
  __syncthreads();
  const int t = blockIdx.x * 256 + tid;
  int key = 0, g = 0;
  unsigned local = 0u;
  if (t < n) {
    g = G == 1 ? 0 : xcd_group(t, nsx, region);
    key = g * kBuckets + cost_rank(cost[t]);
    local = atomicAdd(&cnt[key], 1u);
  }
  __syncthreads();
  for (int i = tid; i < G * kBuckets; i += 256)
    if (cnt[i] != 0u) off[i] = atomicAdd(&base[i], cnt[i]);
  __syncthreads();
  if (t < n) order[(int)(off[key] + local) * G + g] = t;
}

// Single frame: the launch order above with G = kXcdGroups, where every
// workgroup does the scan for itself.  A workgroup forms the
// exclusive prefix sums of each group's bucket histogram in LDS (thread i
// holds 16 consecutive buckets, 32 threads a group), and reserves the
// ranges of its own tiles through the bucket cursors, which start at zero.
// The grid also marks the launch slots past each group's tiles empty (-1).
__global__ __launch_bounds__(256) void plan_place_kernel(const int* cost, int n, int nsx,
                                                         int region, const unsigned* hist,
                                                         unsigned* cursor, int* order,
                                                         int nslots) {
  constexpr int kWords = kXcdGroups * kBuckets;
  constexpr int kPer = kWords / 256;       // buckets per thread
  constexpr int kSeg = kBuckets / kPer;    // threads per group
  static_assert(kWords % (4 * 256) == 0 && kSeg <= 64 && (kSeg & (kSeg - 1)) == 0,
                "bucket layout of the per-workgroup scan");
  __shared__ unsigned pre[kWords];
  __shared__ unsigned cnt[kWords];
  __shared__ unsigned total[kXcdGroups];
  const int tid = threadIdx.x;
  unsigned v[kPer];
  unsigned sum = 0u;
#pragma unroll
  for (int q = 0; q < kPer; q += 4) {
    const uint4 w = *reinterpret_cast<const uint4*>(hist + tid * kPer + q);
    v[q] = w.x;
    v[q + 1] = w.y;
    v[q + 2] = w.z;
    v[q + 3] = w.w;
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) sum += v[q];
  // inclusive scan of the thread sums within each segment of kSeg lanes
  const int seg_lane = __lane_id() & (kSeg - 1);
  unsigned incl = sum;
#pragma unroll
  for (int d = 1; d < kSeg; d <<= 1) {
    const unsigned o = __shfl_up(incl, d, kSeg);
    if (seg_lane >= d) incl += o;
  }
  unsigned run = incl - sum;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    pre[tid * kPer + q] = run;
    cnt[tid * kPer + q] = 0u;
    run += v[q];
  }
  if (seg_lane == kSeg - 1) total[tid / kSeg] = run;
  __syncthreads();
  for (int i = blockIdx.x * 256 + tid; i < nslots; i += gridDim.x * 256)
    if ((unsigned)(i / kXcdGroups) >= total[i % kXcdGroups]) order[i] = -1;
  const int t = blockIdx.x * 256 + tid;
  int key = 0, g = 0;
  unsigned local = 0u;
  if (t < n) {
    g = xcd_group(t, nsx, region);
    key = g * kBuckets + cost_rank(cost[t]);
    local = atomicAdd(&cnt[key], 1u);
  }
  __syncthreads();
  for (int i = tid; i < kWords; i += 256)
    if (cnt[i] != 0u) pre[i] += atomicAdd(&cursor[i], cnt[i]);
  __syncthreads();
  // with counters that started at zero every position is below nslots; the
  // test keeps counters left over from an interrupted frame in bounds
  const unsigned pos = (pre[key] + local) * kXcdGroups + g;
  if (t < n && pos < (unsigned)nslots) order[pos] = t;
}

// Batch class: clear the bucket counters and every request's sample
// counter (one workgroup).
__global__ __launch_bounds__(256) void batch_zero_kernel(BatchDev b) {
  for (int i = threadIdx.x; i < kBuckets; i += 256) b.tile_hist[i] = 0u;
  for (int r = threadIdx.x; r < b.nreq; r += 256)
    if (b.args[r].samples != nullptr) *b.args[r].samples = 0ull;
}

// Batch class: work estimate of every super-tile of every request, and the
// bucket histogram.
__global__ __launch_bounds__(256) void batch_cost_kernel(BatchDev b) {
  __shared__ unsigned h[kBuckets];
  const int tid = threadIdx.x;
  for (int i = tid; i < kBuckets; i += 256) h[i] = 0u;
  __syncthreads();
  const int t = blockIdx.x * 256 + tid;
  if (t < b.ntiles) {
    const int r = batch_request(b.tile_base, b.nreq, t);
    const int c = supertile_cost(b.args[r], t - b.tile_base[r]);
    b.tile_cost[t] = c;
    atomicAdd(&h[cost_rank(c)], 1u);
  }
  __syncthreads();
  for (int i = tid; i < kBuckets; i += 256)
    if (h[i] != 0u) atomicAdd(&b.tile_hist[i], h[i]);
}

// Index of the point that thread t evaluates: the locality order's entry
// when the binning pass chose it, else t.
__device__ __forceinline__ int64_t eval_point(const EvalArgsDev& a, int64_t t) {
  return (a.order != nullptr && *a.use_order != 0u) ? (int64_t)a.order[t] : t;
}

template <int P, int STORE, bool GRAD, bool RAT>
__global__ __launch_bounds__(256) void eval_kernel(EvalArgsDev a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.n) return;
  const int64_t i = eval_point(a, t);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.m.ctrl, a.m.ctrl_bytes);
  const __amdgpu_buffer_rsrc_t rsw = make_rsrc(RAT ? a.m.wctrl : a.m.ctrl,
                                               RAT ? a.m.wctrl_bytes : a.m.ctrl_bytes);
  double u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double x = a.xyz[3 * i + k];
    const double v = (x - a.m.ax[k].lo) * a.m.ax[k].inv_ext;
    u[k] = fmin(fmax(v, 0.0), 1.0);
  }
  int span[3];
  float f, g[3];
  query<P, STORE, GRAD, RAT>(a.m, rs, rsw, u, span, true, f, g);
  a.value[i] = f;
  if (GRAD) {
    a.grad[3 * i + 0] = g[0];
    a.grad[3 * i + 1] = g[1];
    a.grad[3 * i + 2] = g[2];
  }
}

// Value, world gradient and world Hessian at points (non-rational models).
template <int P, int STORE>
__global__ __launch_bounds__(256) void eval_hess_kernel(EvalArgsDev a) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= a.n) return;
  const int64_t i = eval_point(a, t);
  const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.m.ctrl, a.m.ctrl_bytes);
  double u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double x = a.xyz[3 * i + k];
    u[k] = fmin(fmax((x - a.m.ax[k].lo) * a.m.ax[k].inv_ext, 0.0), 1.0);
  }
  int span[3];
  float f, g[3], h[6];
  query_hess<P, STORE>(a.m, rs, u, span, true, f, g, h);
  a.value[i] = f;
  if (a.grad != nullptr) {
    a.grad[3 * i + 0] = g[0];
    a.grad[3 * i + 1] = g[1];
    a.grad[3 * i + 2] = g[2];
  }
  float* o = a.hess + 6 * i;
#pragma unroll
  for (int c = 0; c < 6; ++c) o[c] = h[c];
}

// ---------------------------------------------------------------------------
// locality order of point queries: a radix sort by cell
// ---------------------------------------------------------------------------

// Sort key of a point: its bin, the cell on a 16^3 grid over the box, the
// three 4-bit slab indices interleaved (Morton order, x lowest).  The
// parameter is the one the evaluation forms; u * 16 is exact, so slab j
// holds exactly the parameters in [j/16, (j+1)/16) (and 1 in the last
// slab).
__device__ __forceinline__ unsigned eval_key(const EvalOrderDev& o, int64_t i) {
  constexpr int C = kEvalKeyBits / 3;
  unsigned code = 0u;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double u = fmin(fmax((o.xyz[3 * i + k] - o.lo[k]) * o.inv_ext[k], 0.0), 1.0);
    const unsigned c = (unsigned)min((int)(u * (double)(1 << C)), (1 << C) - 1);
#pragma unroll
    for (int b = 0; b < C; ++b) code |= ((c >> b) & 1u) << (3 * b + k);
  }
  return code;
}
static_assert(kEvalKeyBits == 3 * kEvalBinBits, "the key is the bin");

// Whether to form the keys: always when forced; else kEvalProbeWaves
// waves, spread evenly over the points, each compare the bins of 64
// consecutive points, and the keys are formed when more than one
// neighbouring pair in eight changes bin.  The first count then notes
// whether the keys are out of order (flags[3]); only then do the sorting
// passes run and the evaluation follow the order (flags[1], set by the
// first scan).
constexpr int kEvalProbeWaves = 256;
__device__ __forceinline__ bool eval_form_keys(const EvalOrderDev& o) {
  return o.force != 0 || (uint64_t)o.flags[0] * 8u > (uint64_t)kEvalProbeWaves * 63u;
}

// Lanes of the wave whose digit equals this lane's (among the valid lanes):
// six ballots, one per digit bit.
__device__ __forceinline__ unsigned long long match_digit(unsigned d, bool valid) {
  unsigned long long m = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kEvalDigitBits; ++b) {
    const bool bit = ((d >> b) & 1u) != 0u;
    const unsigned long long bb = __ballot(bit);
    m &= bit ? bb : ~bb;
  }
  return m;
}

// Counters, and the bin bounds of the binned evaluation set to "empty at n".
__global__ __launch_bounds__(256) void eval_order_zero(EvalOrderDev o) {
  if (threadIdx.x < 4) o.flags[threadIdx.x] = 0u;
  if (o.bins)
    for (int b = threadIdx.x; b <= kEvalBins; b += 256) o.bin_start[b] = (int32_t)o.n;
}

// Needs n >= 64 kEvalProbeWaves (the host orders from 2^16 points on).
__global__ __launch_bounds__(256) void eval_order_probe(EvalOrderDev o) {
  const int lane = threadIdx.x & 63;
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t i = (int64_t)w * (o.n / kEvalProbeWaves) + lane;
  const unsigned code = eval_key(o, i);
  const unsigned prev = (unsigned)__shfl_up((int)code, 1, 64);
  const unsigned long long m = __ballot(lane > 0 && prev != code);
  if (lane == 0 && m != 0ull) atomicAdd(&o.flags[0], (unsigned)__popcll(m));
}

// Digit of a key in pass PASS (least significant first).
template <int PASS>
__device__ __forceinline__ unsigned eval_digit(unsigned key) {
  return (key >> (PASS * kEvalDigitBits)) & (unsigned)(kEvalDigits - 1);
}

// Digit counts of workgroup g's points [g C, g C + C) (C = kEvalSortChunk),
// written digit-major (digit d at d * groups + g); each wave adds its
// lanes of one digit at once.  The first pass also forms every point's key
// and notes whether any key is below its predecessor's.
template <int PASS>
__global__ __launch_bounds__(256) void eval_sort_count(EvalOrderDev o) {
  if constexpr (PASS == 0) {
    if (!eval_form_keys(o)) return;
  } else {
    if (o.flags[1] == 0u) return;
  }
  constexpr int J = kEvalSortChunk / 256;
  __shared__ unsigned h[kEvalDigits];
  __shared__ unsigned last[J][4];  // first pass: each wave's last key per round
  __shared__ unsigned h_desc;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid < kEvalDigits) h[tid] = 0u;
  if (tid == 0) h_desc = 0u;
  const int64_t base = (int64_t)blockIdx.x * kEvalSortChunk;
  // the thread's keys first (their loads in flight together)
  unsigned key[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t i = base + j * 256 + tid;
    if constexpr (PASS == 0)
      key[j] = i < o.n ? eval_key(o, i) : 0u;
    else
      key[j] = i < o.n ? (unsigned)o.key[PASS & 1][i] : 0u;
  }
  bool descent = false;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t i = base + j * 256 + tid;
    const bool valid = i < o.n;
    if constexpr (PASS == 0) {
      if (valid) o.key[0][i] = (uint16_t)key[j];
      const unsigned prev = (unsigned)__shfl_up((int)key[j], 1, 64);
      descent |= valid && lane > 0 && key[j] < prev;
      if (lane == 63) last[j][w] = key[j];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int64_t i = base + j * 256 + tid;
    const bool valid = i < o.n;
    if constexpr (PASS == 0) {
      // a wave's first lane against the point before it
      if (lane == 0 && valid && i > 0) {
        const unsigned prev = w > 0 ? last[j][w - 1]
                              : j > 0 ? last[j - 1][3] : eval_key(o, i - 1);
        descent |= key[j] < prev;
      }
    }
    const unsigned d = eval_digit<PASS>(key[j]);
    const unsigned long long m = match_digit(d, valid);
    if (valid && (m >> lane) == 1ull) atomicAdd(&h[d], (unsigned)__popcll(m));
  }
  if constexpr (PASS == 0) {
    if (__ballot(descent) != 0ull && lane == 0) h_desc = 1u;
  }
  __syncthreads();
  if (tid < kEvalDigits) o.hist[(int64_t)tid * o.groups + blockIdx.x] = h[tid];
  // one flag update per workgroup, none once another has set it
  if (PASS == 0 && tid == 0 && h_desc != 0u && o.flags[3] == 0u) atomicOr(&o.flags[3], 1u);
}

__device__ __forceinline__ unsigned wave_inclusive_scan(unsigned v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// Exclusive prefix sum of v over a workgroup of 1024 threads (thread
// order); total receives the sum.  wsum: 16 words of LDS.
__device__ __forceinline__ unsigned block_scan_1024(unsigned v, unsigned* wsum,
                                                    unsigned& total) {
  const int w = threadIdx.x >> 6;
  const unsigned incl = wave_inclusive_scan(v);
  if (__lane_id() == 63) wsum[w] = incl;
  __syncthreads();
  unsigned before = 0u, all = 0u;
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const unsigned x = wsum[k];
    before += k < w ? x : 0u;
    all += x;
  }
  __syncthreads();
  total = all;
  return before + incl - v;
}

// Exclusive prefix sums of the digit counts over the workgroups, in place:
// workgroup d scans digit d's row of `groups` counts, 2048 at a time, and
// records the row's total.  The scatter adds the totals of the smaller
// digits.  The first pass's scan also records whether the points are
// sorted and evaluated in that order (flags[1]).
__global__ __launch_bounds__(256) void eval_sort_scan(EvalOrderDev o, int first) {
  __shared__ unsigned wsum[4];
  const bool use = first ? (eval_form_keys(o) && o.flags[3] != 0u) : o.flags[1] != 0u;
  if (first && blockIdx.x == 0 && threadIdx.x == 0) o.flags[1] = use ? 1u : 0u;
  if (!use) return;
  constexpr int E = 8;  // counts per thread and tile
  unsigned* row = o.hist + (int64_t)blockIdx.x * o.groups;
  const int tid = threadIdx.x, w = tid >> 6;
  unsigned carry = 0u;
  for (int t0 = 0; t0 < o.groups; t0 += 256 * E) {
    unsigned v[E], sum = 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = t0 + tid * E + e;
      v[e] = i < o.groups ? row[i] : 0u;
      sum += v[e];
    }
    const unsigned incl = wave_inclusive_scan(sum);
    if (__lane_id() == 63) wsum[w] = incl;
    __syncthreads();
    unsigned before = carry, all = carry;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      before += k < w ? wsum[k] : 0u;
      all += wsum[k];
    }
    __syncthreads();
    unsigned run = before + incl - sum;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = t0 + tid * E + e;
      if (i < o.groups) row[i] = run;
      run += v[e];
    }
    carry = all;
  }
  if (tid == 0) o.totals[blockIdx.x] = carry;
}

// Stable scatter of workgroup g's points by digit.  The points are first
// ordered by digit in LDS, 256 per round in point order: a wave ranks its
// lanes among those with the same digit, and the waves' counts per digit
// give each wave its first position per digit, after the positions of the
// rounds before.  Then each digit's points, contiguous in LDS, are written
// to the digit's range (coalesced runs).  The workgroup's count of a digit
// is the difference of neighbouring scanned counts.  Pass r reads the keys
// and indices of buffer r % 2 (the first pass: the keys formed by its
// count, indices implicit) and writes buffer (r + 1) % 2.
template <int PASS>
__global__ __launch_bounds__(256) void eval_sort_scatter(EvalOrderDev o) {
  if (o.flags[1] == 0u) return;
  constexpr int J = kEvalSortChunk / 256;
  static_assert(kEvalDigits == 64, "one wave forms the digits' positions");
  __shared__ unsigned lkey[kEvalSortChunk];
  __shared__ int32_t lidx[kEvalSortChunk];
  __shared__ unsigned gbase[kEvalDigits];  // first sorted position of each digit's points
  __shared__ unsigned lbase[kEvalDigits];  // their first position in LDS
  __shared__ unsigned run[kEvalDigits];    // next position in LDS
  __shared__ unsigned wcnt[4][kEvalDigits];
  __shared__ unsigned woff[4][kEvalDigits];
  const uint16_t* kin = o.key[PASS & 1];
  const int32_t* iin = o.idx[PASS & 1];
  uint16_t* kout = o.key[(PASS + 1) & 1];
  int32_t* iout = o.idx[(PASS + 1) & 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int g = blockIdx.x;
  const int64_t base = (int64_t)g * kEvalSortChunk;
  const int cnt = (int)min((int64_t)kEvalSortChunk, o.n - base);
  unsigned key[J];
  int32_t idx[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int l = j * 256 + tid;
    const bool valid = l < cnt;
    key[j] = valid ? kin[base + l] : 0u;
    if constexpr (PASS == 0)
      idx[j] = (int32_t)(base + l);
    else
      idx[j] = valid ? iin[base + l] : 0;
  }
  for (int k = tid; k < 4 * kEvalDigits; k += 256) wcnt[k / kEvalDigits][k % kEvalDigits] = 0u;
  if (tid < kEvalDigits) {
    const unsigned* row = o.hist + (int64_t)tid * o.groups;
    const unsigned t = o.totals[tid];
    const unsigned c = (g + 1 < o.groups ? row[g + 1] : t) - row[g];
    const unsigned lb = wave_inclusive_scan(c) - c;
    lbase[tid] = lb;
    run[tid] = lb;
    gbase[tid] = wave_inclusive_scan(t) - t + row[g];
  }
  __syncthreads();
  const unsigned long long below = (1ull << lane) - 1ull;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const bool valid = j * 256 + tid < cnt;
    const unsigned d = eval_digit<PASS>(key[j]);
    const unsigned long long m = match_digit(d, valid);
    const unsigned rank = (unsigned)__popcll(m & below);
    // the highest lane of each digit's group records the group's size
    if (valid && (m >> lane) == 1ull) wcnt[w][d] = (unsigned)__popcll(m);
    __syncthreads();
    if (tid < kEvalDigits) {
      unsigned r = run[tid];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        woff[v][tid] = r;
        r += wcnt[v][tid];
        wcnt[v][tid] = 0u;
      }
      run[tid] = r;
    }
    __syncthreads();
    if (valid) {
      const unsigned pos = woff[w][d] + rank;
      lkey[pos] = key[j];
      lidx[pos] = idx[j];
    }
  }
  __syncthreads();
  for (int e = tid; e < cnt; e += 256) {
    const unsigned k = lkey[e];
    const unsigned d = eval_digit<PASS>(k);
    const unsigned pos = gbase[d] + ((unsigned)e - lbase[d]);
    kout[pos] = (uint16_t)k;
    iout[pos] = lidx[e];
  }
}

// First sorted position of every non-empty bin (the keys are sorted, as
// formed or by the passes, so a bin starts where the bin number changes).
__global__ __launch_bounds__(256) void eval_bin_mark(EvalOrderDev o) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= o.n) return;
  const uint16_t* key = o.key[o.flags[1] != 0u ? (kEvalPasses & 1) : 0];
  const unsigned k = key[i];
  if (i == 0 || (unsigned)key[i - 1] != k) o.bin_start[k] = (int32_t)i;
}

// Bounds and work items of the bins (one workgroup of 1024 threads, four
// bins each): an empty bin starts where the next non-empty one does (a
// suffix minimum by doubling in LDS), bin b holds
// ceil(count / kEvalItemPoints) work items, and their exclusive prefix sums
// give each bin's first item; flags[2] is the number of items.
__global__ __launch_bounds__(1024) void eval_bin_items(EvalOrderDev o) {
  __shared__ int32_t S[kEvalBins + 1];
  __shared__ unsigned wsum[16];
  const int tid = threadIdx.x;
  for (int b = tid; b <= kEvalBins; b += 1024) S[b] = o.bin_start[b];
  __syncthreads();
  for (int off = 1; off < kEvalBins; off <<= 1) {
    int32_t v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int b = 4 * tid + q;
      v[q] = b + off <= kEvalBins ? min(S[b], S[b + off]) : S[b];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) S[4 * tid + q] = v[q];
    __syncthreads();
  }
  unsigned items[4], sum = 0u;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = 4 * tid + q;
    const unsigned cnt = (unsigned)(S[b + 1] - S[b]);
    items[q] = (cnt + (unsigned)kEvalItemPoints - 1u) / (unsigned)kEvalItemPoints;
    sum += items[q];
  }
  unsigned total;
  unsigned run = block_scan_1024(sum, wsum, total);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int b = 4 * tid + q;
    o.bin_start[b] = S[b];
    o.item_base[b] = (int32_t)run;
    run += items[q];
  }
  if (tid == 0) {
    o.item_base[kEvalBins] = (int32_t)total;
    o.flags[2] = total;
  }
}

// ---------------------------------------------------------------------------
// binned evaluation of point queries from LDS
// ---------------------------------------------------------------------------

// Work item g (see EvalBinDev): its bin (the largest b whose first item is
// at most g; empty bins share their first item with the next bin), its
// share of the bin's points, then the bin's knots, basis-table rows and
// box of control points in LDS.  Each point is evaluated as by
// eval_kernel / eval_hess_kernel, with the same span (searched within the
// slab's span range, which holds it), the same basis arithmetic and the
// same control-point values, so the results are the same bits.
template <int P, int STORE, int MODE>  // MODE 0: value, 1: and gradient, 2: and Hessian
__global__ __launch_bounds__(256) void eval_bin_kernel(EvalArgsDev a, EvalBinDev d) {
  extern __shared__ __align__(16) unsigned char eval_lds[];
  constexpr bool GRAD = MODE >= 1;
  const int g = blockIdx.x;
  if (g >= (int)d.flags[2]) return;
  int lo = 0, hi = kEvalBins;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (d.item_base[mid] <= g)
      lo = mid;
    else
      hi = mid;
  }
  const int bin = lo;
  const int items = d.item_base[bin + 1] - d.item_base[bin];
  const int j = g - d.item_base[bin];
  const int bs = d.bin_start[bin];
  const int64_t cnt = (int64_t)(d.bin_start[bin + 1] - bs);
  const int first = bs + (int)(cnt * j / items);
  const int last = bs + (int)(cnt * (j + 1) / items);

  const int kn = eval_bin_knot_slots(d.nspan);
  double* K = reinterpret_cast<double*>(eval_lds);
  float* T = reinterpret_cast<float*>(K + 3 * kn);
  float* B = T + 3 * d.nspan * d.tstride;
  const int tid = threadIdx.x;
  int slo[3], shi[3], x0[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    int slab = 0;
#pragma unroll
    for (int b = 0; b < kEvalBinBits; ++b) slab |= ((bin >> (3 * b + k)) & 1) << b;
    slo[k] = d.span_lo[k][slab];
    shi[k] = d.span_hi[k][slab];
    x0[k] = slo[k] - a.m.ax[k].p;
  }
  // knots U[slo .. shi+1] and table rows of spans slo .. shi
  for (int e = tid; e < 3 * kn; e += 256) {
    const int k = e / kn, r = e - k * kn;
    if (r <= shi[k] - slo[k] + 1) K[e] = a.m.ax[k].knots[slo[k] + r];
  }
  {
    const int per_axis = d.nspan * d.tstride;
    for (int e = tid; e < 3 * per_axis; e += 256) {
      const int k = e / per_axis, rem = e - k * per_axis;
      const int r = rem / d.tstride, c = rem - r * d.tstride;
      const int ts = table_stride(a.m.ax[k].p);
      if (r <= shi[k] - slo[k] && c < ts)
        T[e] = a.m.ax[k].tab[(size_t)(x0[k] + r) * (size_t)ts + c];
    }
  }
  // box of control points, entries past the grid 0
  const int ex = d.ext[0], ey = d.ext[1], ez = d.ext[2];
  {
    const __amdgpu_buffer_rsrc_t rs = make_rsrc(a.m.ctrl, a.m.ctrl_bytes);
    const int nx = a.m.ax[0].n, ny = a.m.ax[1].n, nz = a.m.ax[2].n;
    const int box = ex * ey * ez;
    // (ix, iy, iz) of element e = tid + 256 r, advanced incrementally
    int iz = tid / (ex * ey);
    int iy = (tid - iz * ex * ey) / ex;
    int ix = tid - iz * ex * ey - iy * ex;
    const int sz = 256 / (ex * ey);
    const int sy = (256 - sz * ex * ey) / ex;
    const int sx = 256 - sz * ex * ey - sy * ex;
    // kStage elements per thread in flight: their loads first, then the
    // LDS stores (element e + 256 j of a batch)
    constexpr int kStage = 8;
    for (int e = tid; e < box; e += 256 * kStage) {
      uint32_t raw[kStage];
      int gi[kStage];
#pragma unroll
      for (int j = 0; j < kStage; ++j) {
        const int gx = x0[0] + ix, gy = x0[1] + iy, gz = x0[2] + iz;
        const bool in = e + 256 * j < box && gx < nx && gy < ny && gz < nz;
        gi[j] = in ? gx + a.m.nx * gy + a.m.nxy * gz : -1;
        const uint32_t off = STORE == 0 ? (uint32_t)max(gi[j], 0) * 4u
                                        : (uint32_t)(max(gi[j], 0) >> 1) * 4u;
        raw[j] = __builtin_amdgcn_raw_buffer_load_b32(rs, off, 0, 0);
        ix += sx;
        iy += sy;
        iz += sz;
        if (ix >= ex) {
          ix -= ex;
          ++iy;
        }
        if (iy >= ey) {
          iy -= ey;
          ++iz;
        }
      }
#pragma unroll
      for (int j = 0; j < kStage; ++j) {
        if (e + 256 * j < box) {
          float v = 0.0f;
          if (gi[j] >= 0) {
            if constexpr (STORE == 0)
              v = __uint_as_float(raw[j]);
            else
              v = (gi[j] & 1) ? h16_hi<STORE>(raw[j]) : h16_lo<STORE>(raw[j]);
          }
          B[e + 256 * j] = v;
        }
      }
    }
  }
  __syncthreads();

  double un[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) un[k] = a.m.ax[k].knots[a.m.ax[k].n];
  const bool uni = a.m.uniform != 0;
  const int pitch_z = ex * ey;
  // sorted by the passes (else the points came in key order)
  const bool permuted = d.flags[1] != 0u;
  for (int t = first + tid; t < last; t += 256) {
    const int64_t i = permuted ? (int64_t)d.order[t] : (int64_t)t;
    double u[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double x = a.xyz[3 * i + k];
      const double v = (x - a.m.ax[k].lo) * a.m.ax[k].inv_ext;
      u[k] = fmin(fmax(v, 0.0), 1.0);
    }
    float N[3][P + 1], dN[3][P + 1], ddN[3][P + 1];
    int off[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const AxisDev& A = a.m.ax[k];
      const double* Kk = K + k * kn - slo[k];  // Kk[s] = U[s] for s in [slo, shi + 1]
      int s;
      if (u[k] >= un[k]) {
        s = A.n - 1;
      } else if (uni) {
        // walked from the cell of u m within the slab's range, which holds
        // the span
        s = min(max(A.p + (int)(u[k] * A.m), slo[k]), shi[k]);
        while (s < shi[k] && Kk[s + 1] <= u[k]) ++s;
        while (s > slo[k] && Kk[s] > u[k]) --s;
      } else {
        int l = slo[k], h = shi[k] + 1;  // U[l] <= u < U[h]
        while (h - l > 1) {
          const int mid = (l + h) >> 1;
          if (Kk[mid] <= u[k])
            l = mid;
          else
            h = mid;
        }
        s = l;
      }
      const float* row = T + (k * d.nspan + (s - slo[k])) * d.tstride;
      if constexpr (MODE == 2)
        query_basis2<P>(A, uni, s, u[k], Kk[s], row, N[k], dN[k], ddN[k]);
      else
        query_basis<P>(A, uni, s, u[k], Kk[s], row, N[k], dN[k]);
      off[k] = s - slo[k];
    }
    const int e0 = off[0] + ex * off[1] + pitch_z * off[2];
    auto fetch = [&](int b, int c, float (&row)[P + 1]) {
      const float* r = B + e0 + b * ex + c * pitch_z;
#pragma unroll
      for (int q = 0; q <= P; ++q) row[q] = r[q];
    };
    float f, gr[3];
    if constexpr (MODE == 2) {
      float h[6];
      contract_hess<P>(N, dN, ddN, fetch, f, gr, h);
      const float sx = a.m.ax[0].gscale, sy = a.m.ax[1].gscale, sz = a.m.ax[2].gscale;
      gr[0] *= sx;
      gr[1] *= sy;
      gr[2] *= sz;
      h[0] *= sx * sx;
      h[1] *= sy * sy;
      h[2] *= sz * sz;
      h[3] *= sx * sy;
      h[4] *= sx * sz;
      h[5] *= sy * sz;
      a.value[i] = f;
      if (a.grad != nullptr) {
        a.grad[3 * i + 0] = gr[0];
        a.grad[3 * i + 1] = gr[1];
        a.grad[3 * i + 2] = gr[2];
      }
      float* o = a.hess + 6 * i;
#pragma unroll
      for (int c = 0; c < 6; ++c) o[c] = h[c];
    } else {
      contract<P, GRAD>(N, dN, fetch, f, gr);
      a.value[i] = f;
      if constexpr (GRAD) {
        a.grad[3 * i + 0] = gr[0] * a.m.ax[0].gscale;
        a.grad[3 * i + 1] = gr[1] * a.m.ax[1].gscale;
        a.grad[3 * i + 2] = gr[2] * a.m.ax[2].gscale;
      }
    }
  }
}

// FP32 FMA issue ceiling: eight independent FMA chains per lane, so that
// the issue rate, not the FMA latency, bounds the loop.  The values stay
// finite (a contraction towards b / (1 - a)); a result is stored only if it
// takes a value it cannot take, so the loop is not removed.
__global__ __launch_bounds__(256) void fma_peak_kernel(float* out, int iters, float a, float b) {
  float x[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) x[k] = (float)(threadIdx.x + k);
#pragma unroll 4
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = fmaf(x[k], a, b);
  }
  float s = 0.0f;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += x[k];
  if (s == -1.0f) out[blockIdx.x] = s;
}

__global__ void zero_counter(unsigned long long* p) {
  if (threadIdx.x == 0) p[0] = 0ull;
}

// Events recorded around the ray-casting kernel alone (not the planning).
hipError_t mark(hipEvent_t ev, hipStream_t st) {
  return ev == nullptr ? hipSuccess : hipEventRecord(ev, st);
}

template <int P, int STORE, bool SHADE, bool FAST, bool EQ, bool CURV = false>
hipError_t launch_brick(const RenderArgsDev& a, hipStream_t st, const KernelEvents& ev) {
  // the frame's counters are zero (plan_init_kernel, then the cost pass of
  // the frame before the previous one)
  const unsigned blocks = (unsigned)((a.ntiles + 255) / 256);
  plan_cost_kernel<<<(unsigned)((a.ntiles + 63) / 64), 256, 0, st>>>(a);
  plan_place_kernel<<<blocks, 256, 0, st>>>(a.tile_cost, a.ntiles, a.nsx, a.region, a.tile_hist,
                                            a.tile_hist + kPlanHistWords, a.tile_order, a.nslots);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = mark(ev.begin, st);
  if (e != hipSuccess) return e;
  if constexpr (CURV) {
    render_brick_kernel<P, STORE, SHADE, FAST, EQ, 4, true><<<a.nslots, 256, a.lds_bytes, st>>>(a);
  } else if (a.lpr == 1) {
    render_brick_kernel<P, STORE, SHADE, FAST, EQ, 1, false><<<a.nslots, 256, a.lds_bytes, st>>>(a);
  } else if (a.lpr == 2) {
    render_brick_kernel<P, STORE, SHADE, FAST, EQ, 2, false><<<a.nslots, 256, a.lds_bytes, st>>>(a);
  } else {
    render_brick_kernel<P, STORE, SHADE, FAST, EQ, 4, false><<<a.nslots, 256, a.lds_bytes, st>>>(a);
  }
  e = hipGetLastError();
  return e == hipSuccess ? mark(ev.end, st) : e;
}

template <int P, int STORE, bool SHADE>
hipError_t launch_render_ps(const RenderArgsDev& a, hipStream_t st, const KernelEvents& ev) {
  if (a.lds_bytes > 0) {
    // EQ: every axis has the kernel's degree P (degree known at compile time)
    const bool eq = a.eq != 0;
    if (a.ctf != nullptr) {
      // curvature transfer function (non-rational models, checked on the
      // host, which plans no bricks above kCurvBrickMaxDegree)
      if constexpr (P <= kCurvBrickMaxDegree) {
        if constexpr (P >= 2) {
          if (a.fast)
            return eq ? launch_brick<P, STORE, SHADE, true, true, true>(a, st, ev)
                      : launch_brick<P, STORE, SHADE, true, false, true>(a, st, ev);
        }
        return eq ? launch_brick<P, STORE, SHADE, false, true, true>(a, st, ev)
                  : launch_brick<P, STORE, SHADE, false, false, true>(a, st, ev);
      } else {
        return hipErrorInvalidValue;
      }
    }
    if constexpr (P >= 2) {
      if (a.fast)
        return eq ? launch_brick<P, STORE, SHADE, true, true>(a, st, ev)
                  : launch_brick<P, STORE, SHADE, true, false>(a, st, ev);
    }
    return eq ? launch_brick<P, STORE, SHADE, false, true>(a, st, ev)
              : launch_brick<P, STORE, SHADE, false, false>(a, st, ev);
  }
  hipError_t e = mark(ev.begin, st);
  if (e != hipSuccess) return e;
  const dim3 grid((a.width + 15) / 16, (a.height + 15) / 16);
  if (a.ctf != nullptr) {
    if (a.m.rational) return hipErrorInvalidValue;   // refused on the host first
    render_global_kernel<P, STORE, SHADE, false, true><<<grid, 256, 0, st>>>(a);
  } else if (a.m.rational) {
    render_global_kernel<P, STORE, SHADE, true, false><<<grid, 256, 0, st>>>(a);
  } else {
    render_global_kernel<P, STORE, SHADE, false, false><<<grid, 256, 0, st>>>(a);
  }
  e = hipGetLastError();
  return e == hipSuccess ? mark(ev.end, st) : e;
}

template <int P, int STORE, bool SHADE, bool FAST, bool EQ>
hipError_t launch_batch_class(const BatchDev& b, int lds_bytes, int lpr, hipStream_t st) {
  const unsigned blocks = (unsigned)((b.ntiles + 255) / 256);
  batch_zero_kernel<<<1, 256, 0, st>>>(b);
  batch_cost_kernel<<<blocks, 256, 0, st>>>(b);
  plan_scan_kernel<<<1, kBuckets, 0, st>>>(b.tile_hist);
  plan_scatter_kernel<1>
      <<<blocks, 256, 0, st>>>(b.tile_cost, b.ntiles, 1, 1, b.tile_hist, b.tile_order);
  if (lpr == 1)
    render_batch_kernel<P, STORE, SHADE, FAST, EQ, 1><<<b.ntiles, 256, lds_bytes, st>>>(b);
  else if (lpr == 2)
    render_batch_kernel<P, STORE, SHADE, FAST, EQ, 2><<<b.ntiles, 256, lds_bytes, st>>>(b);
  else
    render_batch_kernel<P, STORE, SHADE, FAST, EQ, 4><<<b.ntiles, 256, lds_bytes, st>>>(b);
  return hipGetLastError();
}

template <int P, int STORE, bool SHADE>
hipError_t batch_ps(const BatchDev& b, const BatchKey& k, hipStream_t st) {
  if constexpr (P >= 2) {
    if (k.fast)
      return k.eq ? launch_batch_class<P, STORE, SHADE, true, true>(b, k.lds_bytes, k.lpr, st)
                  : launch_batch_class<P, STORE, SHADE, true, false>(b, k.lds_bytes, k.lpr, st);
  }
  return k.eq ? launch_batch_class<P, STORE, SHADE, false, true>(b, k.lds_bytes, k.lpr, st)
              : launch_batch_class<P, STORE, SHADE, false, false>(b, k.lds_bytes, k.lpr, st);
}

template <int P, int STORE>
hipError_t batch_p(const BatchDev& b, const BatchKey& k, hipStream_t st) {
  return k.shading ? batch_ps<P, STORE, true>(b, k, st) : batch_ps<P, STORE, false>(b, k, st);
}

template <int STORE>
hipError_t batch_store(const BatchDev& b, const BatchKey& k, hipStream_t st) {
  switch (k.pmax) {
    case 1: return batch_p<1, STORE>(b, k, st);
    case 2: return batch_p<2, STORE>(b, k, st);
    case 3: return batch_p<3, STORE>(b, k, st);
    case 4: return batch_p<4, STORE>(b, k, st);
    default: return hipErrorInvalidValue;
  }
}

template <int P, int STORE>
hipError_t launch_render_p(const RenderArgsDev& a, hipStream_t st, const KernelEvents& ev) {
  return a.shading ? launch_render_ps<P, STORE, true>(a, st, ev)
                   : launch_render_ps<P, STORE, false>(a, st, ev);
}

template <int P, int STORE>
hipError_t launch_eval_p(const EvalArgsDev& a, hipStream_t st) {
  const unsigned blocks = (unsigned)((a.n + 255) / 256);
  if (a.hess) {
    if (a.m.rational) return hipErrorInvalidValue;   // refused on the host first
    eval_hess_kernel<P, STORE><<<blocks, 256, 0, st>>>(a);
  } else if (a.grad)
    a.m.rational ? eval_kernel<P, STORE, true, true><<<blocks, 256, 0, st>>>(a)
                 : eval_kernel<P, STORE, true, false><<<blocks, 256, 0, st>>>(a);
  else
    a.m.rational ? eval_kernel<P, STORE, false, true><<<blocks, 256, 0, st>>>(a)
                 : eval_kernel<P, STORE, false, false><<<blocks, 256, 0, st>>>(a);
  return hipGetLastError();
}

template <int P, int STORE>
hipError_t launch_eval_bins_p(const EvalArgsDev& a, const EvalBinDev& d, int lds, hipStream_t st) {
  const unsigned blocks = (unsigned)((a.n + kEvalItemPoints - 1) / kEvalItemPoints) + kEvalBins;
  if (a.hess)
    eval_bin_kernel<P, STORE, 2><<<blocks, 256, lds, st>>>(a, d);
  else if (a.grad)
    eval_bin_kernel<P, STORE, 1><<<blocks, 256, lds, st>>>(a, d);
  else
    eval_bin_kernel<P, STORE, 0><<<blocks, 256, lds, st>>>(a, d);
  return hipGetLastError();
}

template <int STORE>
hipError_t dispatch_render(const RenderArgsDev& a, hipStream_t st, const KernelEvents& ev) {
  switch (a.m.pmax) {
    case 1: return launch_render_p<1, STORE>(a, st, ev);
    case 2: return launch_render_p<2, STORE>(a, st, ev);
    case 3: return launch_render_p<3, STORE>(a, st, ev);
    case 4: return launch_render_p<4, STORE>(a, st, ev);
    default: return hipErrorInvalidValue;
  }
}

template <int STORE>
hipError_t dispatch_eval(const EvalArgsDev& a, hipStream_t st) {
  switch (a.m.pmax) {
    case 1: return launch_eval_p<1, STORE>(a, st);
    case 2: return launch_eval_p<2, STORE>(a, st);
    case 3: return launch_eval_p<3, STORE>(a, st);
    case 4: return launch_eval_p<4, STORE>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

// Per-storage entry points, defined in kernels_f32.hip, kernels_bf16.hip
// and kernels_f16.hip (one translation unit each, compiled in parallel).
template <int STORE>
hipError_t render_for_store(const RenderArgsDev& a, hipStream_t st, const KernelEvents& ev) {
  return dispatch_render<STORE>(a, st, ev);
}
template <int STORE>
hipError_t batch_for_store(const BatchDev& b, const BatchKey& k, hipStream_t st) {
  return batch_store<STORE>(b, k, st);
}
template <int STORE>
hipError_t eval_for_store(const EvalArgsDev& a, hipStream_t st) {
  return dispatch_eval<STORE>(a, st);
}
template <int STORE>
hipError_t eval_bins_for_store(const EvalArgsDev& a, const EvalBinDev& d, int lds,
                               hipStream_t st) {
  if (a.m.rational) return hipErrorInvalidValue;  // the host sends these to eval_kernel
  switch (a.m.pmax) {
    case 1: return launch_eval_bins_p<1, STORE>(a, d, lds, st);
    case 2: return launch_eval_bins_p<2, STORE>(a, d, lds, st);
    case 3: return launch_eval_bins_p<3, STORE>(a, d, lds, st);
    case 4: return launch_eval_bins_p<4, STORE>(a, d, lds, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace mfa
