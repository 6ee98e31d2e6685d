// Internal device-side records shared by the C ABI (abi.cpp) and the HIP
// kernels (kernels.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfa {

constexpr int kMaxDegree = 4;
// Largest number of samples one ray may take; the host rejects requests
// whose box diagonal exceeds this many steps.
constexpr int kMaxSamplesPerRay = 1 << 16;
// Lanes that share one ray in the brick ray caster (1, 2 or 4, chosen per
// model; curvature renders always use four); a wave's tile is 8x8, 8x4 or
// 4x4 pixels accordingly.
constexpr int kLanesPerRay = 4;
constexpr int tile_w_of(int lpr) { return lpr == 4 ? 4 : 8; }
constexpr int tile_h_of(int lpr) { return 64 / lpr / tile_w_of(lpr); }

// Launch order of single frames: super-tiles are grouped by square regions
// of `region` x `region` super-tiles into one group per XCD (the hardware
// deals workgroup b to XCD b mod 8), so that each XCD's L2 holds the
// control points of its own regions.  The region side is at most
// kMaxRegion and small enough for about 64 regions, so that every group
// has work on small frames too.
constexpr int kXcdGroups = 8;
constexpr int kMaxRegion = 4;
// Counters of the tile sort (kXcdGroups x 512 buckets).  A frame uses two
// such arrays, the bucket histogram and the bucket cursors; the planning
// scratch of a stream holds two sets, for alternate frames (kPlanWords).
constexpr int kPlanHistWords = kXcdGroups * 512;
constexpr int kPlanWords = 4 * kPlanHistWords;

// Waves per SIMD that the brick ray caster of kernel degree P is compiled
// for (four workgroups of four waves per CU, or three for the variants
// whose registers would otherwise spill; the curvature variants, which also
// carry second derivatives, three at degree 2 on uniform knots and two
// otherwise, up to kCurvBrickMaxDegree), and the LDS one workgroup may use
// at that occupancy (160 KB per CU).  The batch kernel (batch) fits
// general-knot degree 3 with equal degrees in four waves, where the
// single-frame kernel would spill.
__host__ __device__ constexpr int brick_waves_per_simd(int P, bool fast, bool eq,
                                                      bool curv = false, bool batch = false) {
  return curv    ? ((P >= 3 || !fast) ? 2 : 3)
         : batch ? ((P >= 4 || (P == 3 && !fast && !eq)) ? 3 : 4)
                 : ((P >= 4 || (P == 3 && !fast)) ? 3 : 4);
}
// Largest degree whose curvature rendering uses the brick ray caster (its
// registers would spill above; such models use the global-memory kernel).
constexpr int kCurvBrickMaxDegree = 3;
__host__ __device__ constexpr int brick_lds_per_group(int waves) {
  return waves == 2 ? 80 * 1024 : waves == 3 ? 52 * 1024 : 40 * 1024;
}

// Per-span FP32 table of one axis of degree p, for span s (stored at row
// s - p).  With delta = u - U_s (rounded to FP32 once):
//   left[1] = delta,  left[j] = delta + dl[j]   with dl[j] = U_s - U_{s+1-j}, j = 2..p
//   right[j] = dr[j] - delta                    with dr[j] = U_{s+j} - U_s,   j = 1..p
//   inv[q][r] = 1 / (U_{s+r+1} - U_{s+1-q+r}),  q = 1..p, r = 0..q-1
// Layout: dl[2..p], dr[1..p], inv[1][0], inv[2][0..1], ..., inv[p][0..p-1],
// padded to a multiple of 4 floats.
__host__ __device__ constexpr int table_entries(int p) { return 2 * p - 1 + p * (p + 1) / 2; }
__host__ __device__ constexpr int table_stride(int p) { return (table_entries(p) + 3) & ~3; }
__host__ __device__ constexpr int table_dl(int /*p*/, int j) { return j - 2; }
__host__ __device__ constexpr int table_dr(int p, int j) { return (p - 1) + (j - 1); }
__host__ __device__ constexpr int table_inv(int p, int q, int r) {
  return (2 * p - 1) + (q - 1) * q / 2 + r;
}

struct AxisDev {
  const double* knots;  // n + p + 1 knots, FP64
  const float* tab;     // (n - p) rows of table_stride(p) floats
  int32_t n;
  int32_t p;
  double lo;            // box corner along this axis
  double inv_ext;       // 1 / (hi - lo): u = (x - lo) * inv_ext
  double m;             // number of knot spans n - p (as FP64)
  float gscale;         // 1 / (hi - lo) in FP32, world-gradient factor
  float inv_m;          // 1 / (n - p) in FP32
};

struct ModelDev {
  AxisDev ax[3];
  const void* ctrl;     // n0*n1*n2 control points, x fastest
  uint32_t ctrl_bytes;  // size of ctrl in bytes (< 2^31)
  int32_t store;        // 0 FP32, 1 BF16, 2 FP16
  int32_t nx;           // row stride (elements)
  int32_t nxy;          // slice stride (elements)
  int32_t pmax;         // largest degree; kernels are instantiated for it
  int32_t uniform;      // 1: every axis has knots U_{p+k} = k/(n-p) exactly
  int32_t rational;     // 1: ctrl holds w*P and wctrl holds w (homogeneous values)
  uint32_t wctrl_bytes;
  const void* wctrl;    // rational weights in the storage precision, layout of ctrl
};

// Camera, box and step: everything the ray setup of a pixel reads.
struct CamParams {
  double eye[3];
  double F[3], R[3], V[3];
  double cam0, cam1;    // ortho: half_w, half_h; perspective: tan(fov/2), W/H
  double lo[3], hi[3];  // box
  double inv_ext[3];    // 1 / (hi - lo)
  double step;
  int32_t kind;         // 0 ortho, 1 perspective
  int32_t width;
  int32_t height;
  int32_t reserved;
};

struct RenderArgsDev {
  ModelDev m;
  CamParams cam;
  int32_t width;
  int32_t height;
  int32_t ntf;          // transfer-function entries
  int32_t kind;
  const float4* tf;     // ntf RGBA entries
  float tf_lo;          // x = (f - tf_lo) * tf_scale, clamped to [0,1]
  float tf_scale;
  float ert;            // early termination once A > ert
  int32_t shading;
  int32_t shininess;
  float ka, kd, ks;
  float light[3];       // unit vector towards the light
  int32_t fast;         // 1: uniform knots and every degree >= 2 (local-coordinate stepping)
  int32_t eq;           // 1: every axis has degree pmax (degree fixed at compile time)
  float* out;           // width*height*4
  unsigned long long* samples;  // nullable
  // curvature transfer function (nullptr: off): ctf_m x ctf_m RGBA entries,
  // k1 along a row; k = clamp((kappa - ctf_lo) * ctf_scale, 0, 1) (ctf_m - 1)
  const float4* ctf;
  int32_t ctf_m;
  float ctf_lo;
  float ctf_scale;
  // LDS-brick ray marcher (render_brick_kernel); unused by the global caster
  int32_t spr;          // samples per round: each wave stages one brick per round
  int32_t brick_cap;    // floats of LDS per wave for its brick (multiple of 4)
  int32_t lds_knots;    // byte offset of the knot vectors in dynamic LDS (not with fast)
  int32_t lds_bricks;   // byte offset of the bricks in dynamic LDS
  int32_t knot_off[3];  // offset (in doubles) of each axis' knots in LDS
  int32_t lds_bytes;    // dynamic LDS size of one workgroup
  int32_t ntiles;       // super-tiles (2x2 tiles) of the image
  int32_t nsx;          // super-tiles per image row
  int32_t region;       // side of the square regions of the XCD grouping (super-tiles)
  int32_t nslots;       // launch slots: kXcdGroups x the largest group (>= ntiles)
  int32_t lpr;          // lanes per ray (1, 2 or 4)
  int32_t tile_w;       // tile size in pixels (tile_w_of(lpr) x tile_h_of(lpr))
  int32_t tile_h;
  int32_t* tile_cost;   // ntiles work estimates (scratch)
  int32_t* tile_order;  // nslots super-tile indices, -1 for empty slots (scratch)
  unsigned* tile_hist;  // this frame's counters of the tile sort (scratch): histogram,
                        // then cursors (2 x kPlanHistWords, zero before the frame)
  unsigned* tile_clear; // the previous frame's counters, cleared by this frame's planning
};

struct EvalArgsDev {
  ModelDev m;
  double lo[3], hi[3];
  const double* xyz;
  float* value;
  float* grad;          // nullable
  float* hess;          // nullable: n*6 second derivatives (xx, yy, zz, xy, xz, yz)
  int64_t n;
  // locality order (nullable): thread i evaluates point order[i] when
  // *use_order is non-zero (set on the device by the binning pass)
  const int32_t* order;
  const unsigned* use_order;
};

// Locality ordering of large point queries.  A point's key is its bin, its
// cell on a 16^3 grid over the box (16 slabs per axis), the three 4-bit
// slab indices interleaved (Morton order, x lowest).  Unless the keys come
// in order already, the points are sorted by key with a
// least-significant-digit radix sort of two 6-bit digits: each pass counts
// the digits of kEvalSortChunk points per workgroup, scans the counts per
// digit, and scatters the points stably.
constexpr int kEvalBinBits = 4;
constexpr int kEvalSlabs = 1 << kEvalBinBits;
constexpr int kEvalBins = 1 << (3 * kEvalBinBits);
constexpr int kEvalKeyBits = 12;
constexpr int kEvalDigitBits = 6;
constexpr int kEvalDigits = 1 << kEvalDigitBits;
constexpr int kEvalPasses = kEvalKeyBits / kEvalDigitBits;
static_assert(kEvalPasses * kEvalDigitBits == kEvalKeyBits && kEvalKeyBits % 3 == 0,
              "whole digits of a three-axis key");
constexpr int kEvalSortChunk = 4096;
// Work item of the binned evaluation: at most this many points of one bin.
constexpr int kEvalItemPoints = 4096;
// Largest LDS of a binned-evaluation workgroup; models whose slabs need
// more are evaluated by gathers in bin order.
constexpr int kEvalBinMaxLds = 64 * 1024;
struct EvalOrderDev {
  const double* xyz;
  int64_t n;              // <= INT32_MAX
  double lo[3];
  double inv_ext[3];
  int32_t force;          // 1: order whatever the probe finds
  int32_t bins;           // 1: also form the bins' bounds and work items
  int32_t groups;         // sorting workgroups, ceil(n / kEvalSortChunk)
  unsigned* flags;        // [0] bin changes among the probed neighbours,
                          // [1] points sorted by the passes (evaluated in that order),
                          // [2] work items of the bins, [3] keys formed out of order
  uint16_t* key[2];       // n keys each: pass r reads key[r % 2], writes key[(r + 1) % 2]
  int32_t* idx[2];        // n point indices each, likewise (the first pass reads none);
                          // after the last pass idx[kEvalPasses % 2] is the order
  unsigned* hist;         // kEvalDigits * groups digit counts, then their scan per digit
  unsigned* totals;       // kEvalDigits: points per digit
  int32_t* bin_start;     // kEvalBins + 1: first sorted position of each bin
  int32_t* item_base;     // kEvalBins + 1: first work item of each bin
};

// Binned evaluation (non-rational models): work item g takes up to
// kEvalItemPoints points of one bin in the sorted order, stages in LDS the
// knots, basis tables and control points that the bin's windows can touch,
// and evaluates its points from LDS.  Slab j of axis k holds parameters in
// [j/16, (j+1)/16) (the last slab also 1); its points' knot spans lie in
// [span_lo[k][j], span_hi[k][j]].  The staged box of control points starts
// at span_lo - p per axis and has ext[k] = (most spans of a slab) + pmax
// entries (entries past the grid are staged as 0).
struct EvalBinDev {
  const int32_t* order;   // point indices in sorted order (used when flags[1])
  const int32_t* bin_start;
  const int32_t* item_base;
  const unsigned* flags;
  int32_t span_lo[3][kEvalSlabs];
  int32_t span_hi[3][kEvalSlabs];
  int32_t ext[3];
  int32_t nspan;          // most spans of a slab on any axis
  int32_t tstride;        // table row stride in LDS (floats)
};

// The requests of a render batch that share one kernel variant (a class):
// their records in device memory and the class's planning scratch.
struct BatchDev {
  const RenderArgsDev* args;  // nreq request records
  const int32_t* tile_base;   // nreq + 1 prefix sums of the requests' super-tiles
  int32_t nreq;
  int32_t ntiles;             // super-tiles of all requests of the class
  int32_t* tile_cost;         // ntiles work estimates (scratch)
  int32_t* tile_order;        // ntiles class-wide super-tile indices, longest first
  unsigned* tile_hist;        // 512 bucket counters (scratch)
};

// Kernel variant of a batch class and the dynamic LDS of its launch.
struct BatchKey {
  int32_t pmax;
  int32_t store;
  int32_t shading;
  int32_t fast;
  int32_t eq;
  int32_t lpr;
  int32_t lds_bytes;
};

// Optional events recorded on the render stream immediately before and after
// the ray-casting kernel (null: not recorded).
struct KernelEvents {
  hipEvent_t begin = nullptr;
  hipEvent_t end = nullptr;
};

// Device memory of the allocation-free render entry point
// (mfa_render_noalloc): a fixed array per GPU, laid out as the transfer
// function (up to 4096 RGBA entries), the two counter sets of the tile
// sort, then the cost and order arrays of at most kNoAllocMaxSlots launch
// slots.  Every call on a GPU uses the same array.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
constexpr size_t kNoAllocTfOff = 0;
constexpr size_t kNoAllocTfBytes = size_t(4096) * 16;
constexpr size_t kNoAllocCountersOff = kNoAllocTfOff + kNoAllocTfBytes;
constexpr size_t kNoAllocSlotsOff = kNoAllocCountersOff + size_t(kPlanWords) * 4;
constexpr int64_t kNoAllocMaxSlots =
    int64_t((kNoAllocScratchBytes - kNoAllocSlotsOff) / 8) & ~int64_t(63);
static_assert(kNoAllocSlotsOff % 256 == 0, "scratch parts stay 256-byte aligned");

// Device address of that array on the current device (kernels.hip, where
// the array is defined): looked up once per device through the runtime and
// kept; the caller makes `device` current first.
hipError_t noalloc_scratch(int device, void** out);

// Kernel launchers (kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_render(const RenderArgsDev& a, hipStream_t stream, const KernelEvents& ev);
hipError_t launch_render_batch(const BatchDev& b, const BatchKey& k, hipStream_t stream);
hipError_t launch_eval(const EvalArgsDev& a, hipStream_t stream);
hipError_t launch_eval_order(const EvalOrderDev& o, hipStream_t stream);
// Binned evaluation after launch_eval_order with bins = 1; lds_bytes from
// eval_bin_lds_bytes().
hipError_t launch_eval_bins(const EvalArgsDev& a, const EvalBinDev& d, int lds_bytes,
                            hipStream_t stream);
// LDS of a binned-evaluation workgroup: per axis an even number of knot
// slots (at least nspan + 1 doubles), then per axis nspan table rows of
// tstride floats, then the box of control points (FP32).
__host__ __device__ constexpr int eval_bin_knot_slots(int nspan) {
  return (nspan + 2) & ~1;
}
__host__ __device__ constexpr int eval_bin_lds_bytes(int nspan, int tstride, int box) {
  return 3 * eval_bin_knot_slots(nspan) * 8 + 3 * nspan * tstride * 4 + box * 4;
}
// Initial state of a single frame's planning scratch: kPlanWords zero
// counters at hist.
hipError_t launch_plan_init(unsigned* hist, hipStream_t stream);
// FP32 FMA micro-loop: blocks x 256 threads, iters x 8 FMA each
hipError_t launch_fma_peak(float* out, int blocks, int iters, hipStream_t stream);

}  // namespace mfa
