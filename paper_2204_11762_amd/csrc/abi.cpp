// C ABI of the MFA ray-casting library: argument validation, model
// preparation and residency, transfer-function staging and kernel launches.
// The arithmetic of rendering lives in kernels.hip; this file only checks,
// converts and moves data, and fills the launch records.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "mfa_dev.h"
#include "mfa_dvr.h"

namespace {

thread_local std::string g_last_error;

mfa_status fail(mfa_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

std::string hip_msg(const char* what, hipError_t e) {
  return std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
}

constexpr int64_t kMaxCtrlBytes = (int64_t(1) << 31) - 1;
constexpr int64_t kMaxCount = int64_t(1) << 24;  // control points per axis
constexpr int kCtrlPadElems = 16;                // zero padding after the control points
constexpr int64_t kMaxPixels = int64_t(1) << 26;
constexpr int kMaxImageSide = 1 << 15;
constexpr int64_t kMaxEvalPoints = int64_t(1) << 38;
// Requests of one render batch.
constexpr int32_t kMaxBatch = 1 << 16;
// Round lengths (knot spans along the fastest axis per lane's round) that
// mfa_autotune times; 3 is the default.
constexpr double kTuneRoundSpans[] = {1.5, 2.0, 3.0, 4.0, 6.0};
constexpr int32_t kTuneLanes[] = {4, 2, 1};
constexpr size_t kMaxCachedTF = 64;
// Render launches whose kernel duration one timing record holds.
constexpr size_t kMaxTimedLaunches = 1 << 16;

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// --------------------------------------------------------------------------
// validation (host only)
// --------------------------------------------------------------------------

mfa_status check_axis(const mfa_model_desc* d, int k, std::string& msg) {
  const int p = d->degree[k];
  const int64_t n = d->n_ctrl[k];
  const char ax = "xyz"[k];
  if (p < 1 || p > MFA_MAX_DEGREE) {
    msg = std::string("degree of axis ") + ax + " must be in [1, 4]";
    return MFA_ERR_MODEL;
  }
  if (n < p + 1 || n > kMaxCount) {
    msg = std::string("axis ") + ax + ": need p+1 <= n <= 2^24 control points";
    return MFA_ERR_MODEL;
  }
  const double* U = d->knots[k];
  if (U == nullptr) {
    msg = std::string("axis ") + ax + ": null knot vector";
    return MFA_ERR_MODEL;
  }
  const int64_t m = n + p + 1;
  for (int64_t i = 0; i < m; ++i) {
    if (!std::isfinite(U[i])) {
      msg = std::string("axis ") + ax + ": non-finite knot";
      return MFA_ERR_MODEL;
    }
    if (i > 0 && U[i] < U[i - 1]) {
      msg = std::string("axis ") + ax + ": knots must be non-decreasing";
      return MFA_ERR_MODEL;
    }
  }
  for (int i = 0; i <= p; ++i) {
    if (U[i] != 0.0 || U[n + i] != 1.0) {
      msg = std::string("axis ") + ax + ": knot vector must be clamped to [0, 1] (p+1 zeros, p+1 ones)";
      return MFA_ERR_MODEL;
    }
  }
  int64_t run = 0;
  for (int64_t i = p + 1; i < n; ++i) {
    if (!(U[i] > 0.0 && U[i] < 1.0)) {
      msg = std::string("axis ") + ax + ": interior knots must lie in (0, 1)";
      return MFA_ERR_MODEL;
    }
    run = (i > p + 1 && U[i] == U[i - 1]) ? run + 1 : 1;
    if (run > p) {
      msg = std::string("axis ") + ax + ": interior knot multiplicity exceeds the degree";
      return MFA_ERR_MODEL;
    }
  }
  if (!(std::isfinite(d->lo[k]) && std::isfinite(d->hi[k]) && d->lo[k] < d->hi[k])) {
    msg = std::string("axis ") + ax + ": need finite lo < hi";
    return MFA_ERR_MODEL;
  }
  return MFA_OK;
}

mfa_status validate_model(const mfa_model_desc* d, std::string& msg) {
  if (d == nullptr) {
    msg = "null model descriptor";
    return MFA_ERR_INVALID;
  }
  if (d->store != MFA_STORE_F32 && d->store != MFA_STORE_BF16 && d->store != MFA_STORE_F16) {
    msg = "unknown storage precision";
    return MFA_ERR_MODEL;
  }
  for (int k = 0; k < 3; ++k) {
    const mfa_status st = check_axis(d, k, msg);
    if (st != MFA_OK) return st;
  }
  if (d->ctrl == nullptr) {
    msg = "null control points";
    return MFA_ERR_MODEL;
  }
  const int64_t nx = d->n_ctrl[0], ny = d->n_ctrl[1], nz = d->n_ctrl[2];
  const int64_t elem = d->store == MFA_STORE_F32 ? 4 : 2;
  const int pmax = std::max(d->degree[0], std::max(d->degree[1], d->degree[2]));
  // every element index a row load can form, including the zero-weight
  // rows of a lower-degree axis, must stay addressable with 32-bit offsets
  const double reach = double(nx) * double(ny) * double(nz) +
                       double(pmax) * (double(nx) * double(ny) + double(nx) + 1.0) +
                       double(kCtrlPadElems);
  if (reach * double(elem) > double(kMaxCtrlBytes)) {
    msg = "model too large: control points must fit in 2^31 bytes";
    return MFA_ERR_INVALID;
  }
  const int64_t total = nx * ny * nz;
  // stored values: P, or w*P and w for a rational model
  auto storable = [&](double v, const char* what) {
    if (!std::isfinite(v) || !std::isfinite(float(v))) {
      msg = std::string(what) + " must be finite and within FP32 range";
      return false;
    }
    // binary16: float values of magnitude >= 65520 round to infinity
    if (d->store == MFA_STORE_F16 && std::fabs(float(v)) >= 65520.0f) {
      msg = std::string(what) + " must lie within the FP16 range (|x| < 65520)";
      return false;
    }
    return true;
  };
  for (int64_t i = 0; i < total; ++i) {
    if (!storable(d->ctrl[i], "control points")) return MFA_ERR_MODEL;
    if (d->weights != nullptr) {
      const double w = d->weights[i];
      if (!(std::isfinite(w) && w > 0.0)) {
        msg = "rational weights must be finite and positive";
        return MFA_ERR_MODEL;
      }
      // the weight must stay positive after rounding to the storage precision
      if (!storable(w, "rational weights") || !storable(w * d->ctrl[i], "weighted control points"))
        return MFA_ERR_MODEL;
      if (float(w) < FLT_MIN || (d->store == MFA_STORE_F16 && w < 6.2e-5) ||
          (d->store == MFA_STORE_BF16 && w < 1.2e-38)) {
        msg = "rational weights too small for the storage precision";
        return MFA_ERR_MODEL;
      }
    }
  }
  return MFA_OK;
}

bool finite3(const double* v) {
  return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]);
}

struct Frame {
  double F[3], R[3], V[3];
};

// F = unit(target - eye), R = unit(F x up), V = R x F.  Each unit vector is
// x / sqrt(x.x) with the dot product summed left to right.
bool camera_frame(const mfa_camera* c, Frame& fr) {
  double f[3] = {c->target[0] - c->eye[0], c->target[1] - c->eye[1], c->target[2] - c->eye[2]};
  const double lf = std::sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
  if (!(lf > 0.0) || !std::isfinite(lf)) return false;
  for (int k = 0; k < 3; ++k) fr.F[k] = f[k] / lf;
  const double* u = c->up;
  const double r[3] = {fr.F[1] * u[2] - fr.F[2] * u[1], fr.F[2] * u[0] - fr.F[0] * u[2],
                       fr.F[0] * u[1] - fr.F[1] * u[0]};
  const double lr = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  if (!(lr > 0.0) || !std::isfinite(lr)) return false;
  for (int k = 0; k < 3; ++k) fr.R[k] = r[k] / lr;
  fr.V[0] = fr.R[1] * fr.F[2] - fr.R[2] * fr.F[1];
  fr.V[1] = fr.R[2] * fr.F[0] - fr.R[0] * fr.F[2];
  fr.V[2] = fr.R[0] * fr.F[1] - fr.R[1] * fr.F[0];
  return true;
}

mfa_status validate_render(const mfa_camera* c, const mfa_tf* tf, const mfa_render_params* p,
                           std::string& msg) {
  if (c == nullptr || tf == nullptr || p == nullptr) {
    msg = "null camera, transfer function or parameters";
    return MFA_ERR_INVALID;
  }
  if (c->kind != MFA_CAMERA_ORTHO && c->kind != MFA_CAMERA_PERSP) {
    msg = "unknown camera kind";
    return MFA_ERR_INVALID;
  }
  if (c->width < 1 || c->height < 1 || c->width > kMaxImageSide || c->height > kMaxImageSide ||
      int64_t(c->width) * int64_t(c->height) > kMaxPixels) {
    msg = "image size must be positive, at most 32768 per side and 2^26 pixels";
    return MFA_ERR_INVALID;
  }
  if (!finite3(c->eye) || !finite3(c->target) || !finite3(c->up)) {
    msg = "camera vectors must be finite";
    return MFA_ERR_INVALID;
  }
  Frame fr;
  if (!camera_frame(c, fr)) {
    msg = "degenerate camera (eye == target or up parallel to the view axis)";
    return MFA_ERR_INVALID;
  }
  if (c->kind == MFA_CAMERA_PERSP) {
    if (!(c->fov_y_deg > 0.0 && c->fov_y_deg < 180.0)) {
      msg = "perspective field of view must be in (0, 180) degrees";
      return MFA_ERR_INVALID;
    }
  } else if (!(c->ortho_half_w > 0.0 && c->ortho_half_h > 0.0 && std::isfinite(c->ortho_half_w) &&
               std::isfinite(c->ortho_half_h))) {
    msg = "orthographic half extents must be positive";
    return MFA_ERR_INVALID;
  }
  if (tf->n < 2 || tf->n > MFA_MAX_TF || tf->rgba == nullptr) {
    msg = "transfer function needs 2..4096 entries";
    return MFA_ERR_INVALID;
  }
  if (!(std::isfinite(tf->v_lo) && std::isfinite(tf->v_hi) && tf->v_lo < tf->v_hi)) {
    msg = "transfer function range needs finite v_lo < v_hi";
    return MFA_ERR_INVALID;
  }
  for (int i = 0; i < 4 * tf->n; ++i) {
    if (!std::isfinite(tf->rgba[i])) {
      msg = "transfer function entries must be finite";
      return MFA_ERR_INVALID;
    }
    if (i % 4 == 3 && !(tf->rgba[i] >= 0.0f && tf->rgba[i] <= 1.0f)) {
      msg = "transfer function opacities must lie in [0, 1]";
      return MFA_ERR_INVALID;
    }
  }
  if (!(p->step > 0.0) || !std::isfinite(p->step)) {
    msg = "step must be positive";
    return MFA_ERR_INVALID;
  }
  if (!std::isfinite(p->ert_alpha)) {
    msg = "ert_alpha must be finite";
    return MFA_ERR_INVALID;
  }
  if ((p->shading != 0 && p->shading != 1) || (p->headlight != 0 && p->headlight != 1)) {
    msg = "shading and headlight must be 0 or 1";
    return MFA_ERR_INVALID;
  }
  if (p->shininess < 0 || p->shininess > 256) {
    msg = "shininess must be in [0, 256]";
    return MFA_ERR_INVALID;
  }
  if (!std::isfinite(p->ka) || !std::isfinite(p->kd) || !std::isfinite(p->ks)) {
    msg = "lighting coefficients must be finite";
    return MFA_ERR_INVALID;
  }
  if (!p->headlight) {
    const double* l = p->light_dir;
    if (!finite3(l) || !(l[0] * l[0] + l[1] * l[1] + l[2] * l[2] > 0.0)) {
      msg = "light direction must be finite and non-zero";
      return MFA_ERR_INVALID;
    }
  }
  return MFA_OK;
}

// --------------------------------------------------------------------------
// model preparation
// --------------------------------------------------------------------------

uint16_t to_bf16(double x) {
  const float f = float(x);  // round to nearest even
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even on the upper half
  return uint16_t(u >> 16);
}

// IEEE binary16 encoding of float(x), rounded to nearest even (subnormals
// included; magnitudes that round above 65504 give infinity, which the
// model check refuses).
uint16_t to_f16(double x) {
  const float f = float(x);
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t sign = (u >> 16) & 0x8000u;
  const int e32 = int((u >> 23) & 0xFFu);
  const uint32_t man = u & 0x7FFFFFu;
  if (e32 == 0xFF) return uint16_t(sign | 0x7C00u);
  const int e = e32 - 127 + 15;
  if (e >= 31) return uint16_t(sign | 0x7C00u);
  if (e >= 1) {
    uint32_t h = (uint32_t(e) << 10) | (man >> 13);
    const uint32_t rem = man & 0x1FFFu;
    if (rem > 0x1000u || (rem == 0x1000u && (h & 1u))) ++h;  // a carry may raise the exponent
    return uint16_t(sign | h);
  }
  if (e32 == 0 || e < -10) return uint16_t(sign);
  const uint32_t m = man | 0x800000u;
  const int shift = 14 - e;
  uint32_t q = m >> shift;
  const uint32_t rem = m & ((1u << shift) - 1u);
  const uint32_t halfway = 1u << (shift - 1);
  if (rem > halfway || (rem == halfway && (q & 1u))) ++q;
  return uint16_t(sign | q);
}

// Per-span table rows (layout in mfa_dev.h), computed in FP64 and rounded
// once to FP32.  Empty spans (never located) get zero rows.
void build_table(const double* U, int64_t n, int p, float* out) {
  const int S = mfa::table_stride(p);
  for (int64_t s = p; s < n; ++s) {
    float* row = out + (s - p) * S;
    std::memset(row, 0, sizeof(float) * S);
    if (!(U[s] < U[s + 1])) continue;
    for (int j = 2; j <= p; ++j) row[mfa::table_dl(p, j)] = float(U[s] - U[s + 1 - j]);
    for (int j = 1; j <= p; ++j) row[mfa::table_dr(p, j)] = float(U[s + j] - U[s]);
    for (int q = 1; q <= p; ++q)
      for (int r = 0; r < q; ++r)
        row[mfa::table_inv(p, q, r)] = float(1.0 / (U[s + r + 1] - U[s + 1 - q + r]));
  }
}

struct DeviceModel {
  void* mem = nullptr;
  int64_t bytes = 0;
  mfa::ModelDev md{};
  double lo[3], hi[3];
  int64_t nknots[3];
  int64_t batch_refs = 0;  // live batches that render this model
  double round_spans = 3.0;  // knot spans along the fastest axis per lane's round (tunable)
  int32_t lanes_per_ray = mfa::kLanesPerRay;  // lanes sharing a ray (tunable: 1, 2 or 4)
  // binned point queries: the slabs' span ranges and LDS boxes (pointers
  // set per call), and the LDS of a workgroup (0: not binned, evaluated by
  // gathers in bin order)
  mfa::EvalBinDev bins{};
  int32_t bin_lds_bytes = 0;
};

// LDS plan of the brick ray caster for one request: transfer function,
// knots (general path only), then one brick per wave.  Workgroups are sized for four per CU;
// requests whose tables leave too little room use the global-memory
// fallback kernel (lds_bytes = 0).
constexpr int kMinBrick = 512;

void plan_bricks(const DeviceModel& dm, int ntf, double step, bool curv, bool batch,
                 mfa::RenderArgsDev& a) {
  const int tf_bytes = ntf * 16;
  int knot_doubles = 0;
  for (int k = 0; k < 3; ++k) {
    a.knot_off[k] = knot_doubles;
    // uniform knots are implied by their index on the fast path
    if (!a.fast) knot_doubles += int(dm.nknots[k]);
  }
  const int knot_bytes = (knot_doubles * 8 + 15) & ~15;
  if (curv && dm.md.pmax > mfa::kCurvBrickMaxDegree) {
    // curvature above this degree: the global-memory kernel
    a.lds_bytes = 0;
    a.spr = 0;
    a.brick_cap = 0;
    return;
  }
  const int lds_budget =
      mfa::brick_lds_per_group(
          mfa::brick_waves_per_simd(dm.md.pmax, a.fast != 0, a.eq != 0, curv, batch));
  const int rest = lds_budget - tf_bytes - knot_bytes;
  const int cap = (rest / (4 * 4)) & ~3;
  if (cap < kMinBrick) {
    a.lds_bytes = 0;
    a.spr = 0;
    a.brick_cap = 0;
    return;
  }
  a.lds_knots = tf_bytes;
  a.lds_bricks = tf_bytes + knot_bytes;
  a.brick_cap = cap;
  a.lds_bytes = tf_bytes + knot_bytes + 4 * cap * 4;
  // about round_spans knot spans along the worst axis per lane's round
  double cells = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double span_len = (dm.hi[k] - dm.lo[k]) / dm.md.ax[k].m;
    cells = std::max(cells, step / span_len);
  }
  const int spr = cells > 0.0 ? int(dm.round_spans * a.lpr / cells) : 64;
  a.spr = std::max(4, std::min(64, spr));
}

struct TFEntry {
  std::vector<float> host;
  float4* dev = nullptr;
};

uint64_t fnv1a(const void* p, size_t n) {
  const unsigned char* b = static_cast<const unsigned char*>(p);
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= b[i];
    h *= 1099511628211ull;
  }
  return h;
}

class DeviceGuard {
 public:
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    ok_ = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    if (prev_ >= 0) (void)hipSetDevice(prev_);
  }
  bool ok() const { return ok_; }

 private:
  int prev_ = -1;
  bool ok_ = false;
};

}  // namespace

// A prepared render batch: one device allocation holding the requests'
// kernel records, transfer-function tables and planning scratch, grouped by
// kernel variant; requests that need the global-memory kernel are launched
// one by one from host copies of their records.
struct RenderBatch {
  void* mem = nullptr;
  int64_t bytes = 0;
  std::vector<std::pair<mfa::BatchKey, mfa::BatchDev>> classes;
  std::vector<mfa::RenderArgsDev> single;
  std::vector<int64_t> models;
};

// Planning scratch of one stream: cost and order arrays of `tiles` entries
// each (launch slots), then two sets of bucket counters (kPlanWords).
// Frames alternate between the sets (`parity` names the next frame's), and
// each frame clears the set of the frame before it, so the next frame's set
// is zero.  An init launch clears both on a fresh buffer (ready = false); a
// frame whose launches fail part-way clears `ready`.
struct PlanScratch {
  void* mem = nullptr;
  int64_t tiles = 0;
  bool ready = false;
  int parity = 0;
};
// Point-query locality scratch of one stream: bins, order, counters.
struct EvalScratch {
  void* mem = nullptr;
  int64_t points = 0;
};
// Layout of the ordering scratch for a capacity of `points` points: the
// counters, the bins' starts and first work items, the digit counts of the
// sorting workgroups, then the two buffers of keys and of point indices.
struct EvalLayout {
  size_t flags, totals, bin_start, item_base, hist, key0, key1, idx0, idx1, bytes;
};
EvalLayout eval_layout(int64_t points) {
  EvalLayout l{};
  const int64_t groups = (points + mfa::kEvalSortChunk - 1) / mfa::kEvalSortChunk;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t at = off;
    off = (off + bytes + 255) & ~size_t(255);
    return at;
  };
  l.flags = take(64 * 4);
  l.totals = take(size_t(mfa::kEvalDigits) * 4);
  l.bin_start = take(size_t(mfa::kEvalBins + 1) * 4);
  l.item_base = take(size_t(mfa::kEvalBins + 1) * 4);
  l.hist = take(size_t(mfa::kEvalDigits) * size_t(groups) * 4);
  l.key0 = take(size_t(points) * 2);
  l.key1 = take(size_t(points) * 2);
  l.idx0 = take(size_t(points) * 4);
  l.idx1 = take(size_t(points) * 4);
  l.bytes = off;
  return l;
}
// Knot span of u on a clamped knot vector U with n control points and
// degree p: the largest s in [p, n-1] with U[s] <= u (n-1 from U[n] on),
// as the kernels find it.
int64_t host_span(const double* U, int64_t n, int p, double u) {
  if (u >= U[n]) return n - 1;
  int64_t lo = p, hi = n;
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (U[mid] <= u)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}
// Point queries from this many points on are sorted by bin on the device
// if the model's gathers would miss the caches: when sqrt(control-point
// bytes) * (p+1)^3 reaches kEvalOrderScore.  Below it the control points
// stay cached and ordering costs more than it saves (2^24 random points
// with the gathers in bin order: 32^3 at degree 1 took 0.026 ns per query
// unordered against 0.070 ordered; 128^3 at degree 4 0.358 against 0.144).
// Sorted points are evaluated bin by bin from LDS where the model's slab
// boxes fit (non-rational models), else gathered in bin order.
constexpr int64_t kEvalOrderMin = int64_t(1) << 16;
constexpr double kEvalOrderScore = 4.0e4;
constexpr size_t kMaxPlanStreams = 16;

struct mfa_ctx {
  int device = 0;
  int64_t budget = 0;
  int64_t used = 0;
  int64_t next_id = 1;
  // device address of the allocation-free entry point's fixed array on
  // this context's GPU (looked up when the context is created)
  void* scratch = nullptr;
  std::unordered_map<int64_t, DeviceModel> models;
  std::unordered_map<int64_t, RenderBatch> batches;
  std::unordered_map<uint64_t, std::vector<TFEntry>> tfs;
  size_t n_tf = 0;
  // planning scratch by stream: renders on one stream are ordered by it,
  // renders on different streams never share planning space
  std::unordered_map<void*, PlanScratch> plans;
  // point-query ordering scratch by stream, for the same reason
  std::unordered_map<void*, EvalScratch> evals;
  // kernel timing: event pairs, the first `timed` of which are recorded
  bool timing = false;
  std::vector<mfa::KernelEvents> events;
  size_t timed = 0;

  void free_plans() {
    for (auto& kv : plans) (void)hipFree(kv.second.mem);
    plans.clear();
  }

  void free_evals() {
    for (auto& kv : evals) (void)hipFree(kv.second.mem);
    evals.clear();
  }

  void free_tfs() {
    for (auto& kv : tfs)
      for (auto& e : kv.second) (void)hipFree(e.dev);
    tfs.clear();
    n_tf = 0;
  }
};

namespace {

// Device copy of a transfer-function table, cached by content.  Entries are
// never modified; when the cache is full the device is synchronised before
// the old entries are released.
mfa_status tf_device(mfa_ctx* ctx, const mfa_tf* tf, float4** out) {
  const size_t nfl = size_t(tf->n) * 4;
  const uint64_t h = fnv1a(tf->rgba, nfl * sizeof(float));
  auto it = ctx->tfs.find(h);
  if (it != ctx->tfs.end()) {
    for (auto& e : it->second) {
      if (e.host.size() == nfl && std::memcmp(e.host.data(), tf->rgba, nfl * sizeof(float)) == 0) {
        *out = e.dev;
        return MFA_OK;
      }
    }
  }
  if (ctx->n_tf >= kMaxCachedTF) {
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("hipDeviceSynchronize", e));
    ctx->free_tfs();
  }
  TFEntry ent;
  ent.host.assign(tf->rgba, tf->rgba + nfl);
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&ent.dev), nfl * sizeof(float));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MFA_ERR_NOMEM, hip_msg("hipMalloc (transfer function)", e));
  }
  e = hipMemcpy(ent.dev, ent.host.data(), nfl * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(ent.dev);
    return fail(MFA_ERR_DEVICE, hip_msg("hipMemcpy (transfer function)", e));
  }
  *out = ent.dev;
  ctx->tfs[h].push_back(std::move(ent));
  ctx->n_tf += 1;
  return MFA_OK;
}

// The planning scratch of `stream`, grown to at least `tiles` launch slots,
// and its arrays attached to the records `a` (the counters are attached
// per launch, by plan_counters).  A buffer that must grow, or the whole set
// once it holds kMaxPlanStreams streams, may still be read by enqueued
// kernels, so the device is synchronised before release.
mfa_status attach_plan(mfa_ctx* ctx, void* stream, int64_t tiles, mfa::RenderArgsDev* a, int na,
                       PlanScratch** out) {
  auto it = ctx->plans.find(stream);
  if (it == ctx->plans.end() || it->second.tiles < tiles) {
    const bool grow = it != ctx->plans.end();
    if (grow || ctx->plans.size() >= kMaxPlanStreams) {
      const hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("hipDeviceSynchronize", e));
      if (grow) {
        (void)hipFree(it->second.mem);
        ctx->plans.erase(it);
      } else {
        ctx->free_plans();
      }
    }
    PlanScratch ps;
    // whole groups of 64 slots keep the counters 256-byte aligned
    const int64_t slots = (tiles + 63) & ~int64_t(63);
    const size_t bytes = size_t(slots) * 8 + size_t(mfa::kPlanWords) * 4;
    const hipError_t e = hipMalloc(&ps.mem, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(MFA_ERR_NOMEM, hip_msg("hipMalloc (tile queue)", e));
    }
    ps.tiles = slots;
    it = ctx->plans.emplace(stream, ps).first;
  }
  int32_t* base = static_cast<int32_t*>(it->second.mem);
  const int64_t n = it->second.tiles;
  if (!it->second.ready) {
    const hipError_t e = mfa::launch_plan_init(reinterpret_cast<unsigned*>(base + 2 * n),
                                               static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("tile queue init", e));
    it->second.ready = true;
    it->second.parity = 0;
  }
  for (int i = 0; i < na; ++i) {
    a[i].tile_cost = base;
    a[i].tile_order = base + n;
  }
  *out = &it->second;
  return MFA_OK;
}

// The counter sets of the next frame planned in `ps`, attached to `a`.
void plan_counters(PlanScratch& ps, mfa::RenderArgsDev& a) {
  unsigned* c = reinterpret_cast<unsigned*>(static_cast<int32_t*>(ps.mem) + 2 * ps.tiles);
  a.tile_hist = c + ps.parity * 2 * mfa::kPlanHistWords;
  a.tile_clear = c + (1 - ps.parity) * 2 * mfa::kPlanHistWords;
  ps.parity ^= 1;
}

// After a failed launch the planning scratch of `stream` may be left part-way
// through a frame: the next frame initialises it again.
void plan_unready(mfa_ctx* ctx, void* stream) {
  auto it = ctx->plans.find(stream);
  if (it != ctx->plans.end()) it->second.ready = false;
}

// The ordering scratch of `stream`, grown to at least `points` points, laid
// out in `o` (counters first, then the order, then the bins).  As for the
// planning scratch, a buffer that must be released may still be read by
// enqueued kernels, so the device is synchronised first.
mfa_status attach_eval(mfa_ctx* ctx, void* stream, int64_t points, mfa::EvalOrderDev& o) {
  auto it = ctx->evals.find(stream);
  if (it == ctx->evals.end() || it->second.points < points) {
    const bool grow = it != ctx->evals.end();
    if (grow || ctx->evals.size() >= kMaxPlanStreams) {
      const hipError_t e = hipDeviceSynchronize();
      if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("hipDeviceSynchronize", e));
      if (grow) {
        (void)hipFree(it->second.mem);
        ctx->evals.erase(it);
      } else {
        ctx->free_evals();
      }
    }
    EvalScratch es;
    const hipError_t e = hipMalloc(&es.mem, eval_layout(points).bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return fail(MFA_ERR_NOMEM, hip_msg("hipMalloc (point order)", e));
    }
    es.points = points;
    it = ctx->evals.emplace(stream, es).first;
  }
  const EvalLayout l = eval_layout(it->second.points);
  unsigned char* base = static_cast<unsigned char*>(it->second.mem);
  o.flags = reinterpret_cast<unsigned*>(base + l.flags);
  o.totals = reinterpret_cast<unsigned*>(base + l.totals);
  o.bin_start = reinterpret_cast<int32_t*>(base + l.bin_start);
  o.item_base = reinterpret_cast<int32_t*>(base + l.item_base);
  o.hist = reinterpret_cast<unsigned*>(base + l.hist);
  o.key[0] = reinterpret_cast<uint16_t*>(base + l.key0);
  o.key[1] = reinterpret_cast<uint16_t*>(base + l.key1);
  o.idx[0] = reinterpret_cast<int32_t*>(base + l.idx0);
  o.idx[1] = reinterpret_cast<int32_t*>(base + l.idx1);
  return MFA_OK;
}

}  // namespace

extern "C" {

const char* mfa_last_error(void) { return g_last_error.c_str(); }

const char* mfa_version(void) { return "mfa-dvr-gfx950 0.1"; }

mfa_status mfa_validate_model(const mfa_model_desc* desc) {
  g_last_error.clear();
  std::string msg;
  const mfa_status st = validate_model(desc, msg);
  if (st != MFA_OK) return fail(st, msg);
  return MFA_OK;
}

mfa_status mfa_validate_render(const mfa_camera* camera, const mfa_tf* tf,
                               const mfa_render_params* params) {
  g_last_error.clear();
  std::string msg;
  const mfa_status st = validate_render(camera, tf, params, msg);
  if (st != MFA_OK) return fail(st, msg);
  return MFA_OK;
}

mfa_status mfa_create(int32_t device, mfa_ctx** ctx_out) {
  g_last_error.clear();
  if (ctx_out == nullptr) return fail(MFA_ERR_INVALID, "null ctx_out");
  int count = 0;
  const hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("hipGetDeviceCount", e));
  if (device < 0 || device >= count) return fail(MFA_ERR_DEVICE, "no such HIP device");
  DeviceGuard g(device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  // set-up of the allocation-free entry point: its array's address on this
  // device, with the device current
  void* scratch = nullptr;
  const hipError_t es = mfa::noalloc_scratch(device, &scratch);
  if (es != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("scratch address", es));
  mfa_ctx* ctx = new mfa_ctx();
  ctx->device = device;
  ctx->scratch = scratch;
  *ctx_out = ctx;
  return MFA_OK;
}

mfa_status mfa_destroy(mfa_ctx* ctx) {
  g_last_error.clear();
  if (ctx == nullptr) return MFA_OK;
  mfa_status st = MFA_OK;
  {
    DeviceGuard g(ctx->device);
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) st = fail(MFA_ERR_DEVICE, hip_msg("hipDeviceSynchronize", e));
    for (auto& kv : ctx->batches) (void)hipFree(kv.second.mem);
    ctx->batches.clear();
    for (auto& kv : ctx->models) (void)hipFree(kv.second.mem);
    ctx->models.clear();
    ctx->free_tfs();
    ctx->free_plans();
    ctx->free_evals();
    for (auto& ev : ctx->events) {
      (void)hipEventDestroy(ev.begin);
      (void)hipEventDestroy(ev.end);
    }
    ctx->events.clear();
  }
  delete ctx;
  return st;
}

mfa_status mfa_set_memory_budget(mfa_ctx* ctx, int64_t bytes) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  if (bytes < 0) return fail(MFA_ERR_INVALID, "negative budget");
  ctx->budget = bytes;
  return MFA_OK;
}

mfa_status mfa_model_upload(mfa_ctx* ctx, const mfa_model_desc* d, int64_t* model_out) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  if (model_out == nullptr) return fail(MFA_ERR_INVALID, "null model_out");
  std::string msg;
  const mfa_status st = validate_model(d, msg);
  if (st != MFA_OK) return fail(st, msg);

  const int64_t n[3] = {d->n_ctrl[0], d->n_ctrl[1], d->n_ctrl[2]};
  const int64_t total = n[0] * n[1] * n[2];
  const size_t elem = d->store == MFA_STORE_F32 ? 4 : 2;
  size_t off_knots[3], off_tab[3], off = 0;
  for (int k = 0; k < 3; ++k) {
    off_knots[k] = off;
    off = align256(off + sizeof(double) * size_t(n[k] + d->degree[k] + 1));
  }
  for (int k = 0; k < 3; ++k) {
    off_tab[k] = off;
    off = align256(off + sizeof(float) * size_t(n[k] - d->degree[k]) *
                             size_t(mfa::table_stride(d->degree[k])));
  }
  const size_t off_ctrl = off;
  const size_t ctrl_bytes = elem * size_t(total + kCtrlPadElems);
  const bool rational = d->weights != nullptr;
  const size_t off_w = align256(off_ctrl + ctrl_bytes);
  const size_t bytes = rational ? align256(off_w + ctrl_bytes) : off_w;

  if (ctx->budget > 0 && ctx->used + int64_t(bytes) > ctx->budget)
    return fail(MFA_ERR_NOMEM, "model exceeds the context's memory budget");

  std::vector<unsigned char> host(bytes, 0);
  for (int k = 0; k < 3; ++k) {
    std::memcpy(host.data() + off_knots[k], d->knots[k],
                sizeof(double) * size_t(n[k] + d->degree[k] + 1));
    build_table(d->knots[k], n[k], d->degree[k],
                reinterpret_cast<float*>(host.data() + off_tab[k]));
  }
  // stored plane(s): P, or w*P (homogeneous numerator) and w
  auto store_plane = [&](size_t off_plane, auto value) {
    if (d->store == MFA_STORE_F32) {
      float* c = reinterpret_cast<float*>(host.data() + off_plane);
      for (int64_t i = 0; i < total; ++i) c[i] = float(value(i));
    } else {
      uint16_t* c = reinterpret_cast<uint16_t*>(host.data() + off_plane);
      for (int64_t i = 0; i < total; ++i)
        c[i] = d->store == MFA_STORE_BF16 ? to_bf16(value(i)) : to_f16(value(i));
    }
  };
  if (rational) {
    store_plane(off_ctrl, [&](int64_t i) { return d->weights[i] * d->ctrl[i]; });
    store_plane(off_w, [&](int64_t i) { return d->weights[i]; });
  } else {
    store_plane(off_ctrl, [&](int64_t i) { return d->ctrl[i]; });
  }

  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MFA_ERR_NOMEM, hip_msg("hipMalloc (model)", e));
  }
  e = hipMemcpy(mem, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return fail(MFA_ERR_DEVICE, hip_msg("hipMemcpy (model)", e));
  }

  DeviceModel dm;
  dm.mem = mem;
  dm.bytes = int64_t(bytes);
  unsigned char* base = static_cast<unsigned char*>(mem);
  int pmax = 0;
  int uniform = 1;
  for (int k = 0; k < 3; ++k) {
    mfa::AxisDev& A = dm.md.ax[k];
    A.knots = reinterpret_cast<const double*>(base + off_knots[k]);
    A.tab = reinterpret_cast<const float*>(base + off_tab[k]);
    A.n = int32_t(n[k]);
    A.p = d->degree[k];
    A.lo = d->lo[k];
    A.inv_ext = 1.0 / (d->hi[k] - d->lo[k]);
    A.m = double(n[k] - d->degree[k]);
    A.gscale = float(1.0 / (d->hi[k] - d->lo[k]));
    A.inv_m = float(1.0 / A.m);
    dm.lo[k] = d->lo[k];
    dm.hi[k] = d->hi[k];
    dm.nknots[k] = n[k] + d->degree[k] + 1;
    pmax = std::max(pmax, int(A.p));
    // uniform knot vector: U_{p+j} = j / (n-p) exactly, j = 0..n-p
    const int64_t m = n[k] - d->degree[k];
    for (int64_t j = 0; j <= m && uniform; ++j)
      if (d->knots[k][d->degree[k] + j] != double(j) / double(m)) uniform = 0;
  }
  dm.md.uniform = uniform;
  dm.md.ctrl = base + off_ctrl;
  dm.md.ctrl_bytes = uint32_t(ctrl_bytes);
  dm.md.rational = rational ? 1 : 0;
  dm.md.wctrl = rational ? base + off_w : nullptr;
  dm.md.wctrl_bytes = rational ? uint32_t(ctrl_bytes) : 0u;
  dm.md.store = d->store;
  dm.md.nx = int32_t(n[0]);
  dm.md.nxy = int32_t(n[0] * n[1]);
  dm.md.pmax = pmax;
  // slab span ranges of the binned point queries: slab j of an axis holds
  // the parameters in [j/16, (j+1)/16), the last one also 1
  {
    mfa::EvalBinDev& bd = dm.bins;
    int nspan = 0;
    for (int k = 0; k < 3; ++k) {
      int most = 0;
      for (int j = 0; j < mfa::kEvalSlabs; ++j) {
        const int64_t lo_s = host_span(d->knots[k], n[k], d->degree[k],
                                       double(j) / double(mfa::kEvalSlabs));
        const int64_t hi_s = j + 1 == mfa::kEvalSlabs
                                 ? n[k] - 1
                                 : host_span(d->knots[k], n[k], d->degree[k],
                                             double(j + 1) / double(mfa::kEvalSlabs));
        bd.span_lo[k][j] = int32_t(lo_s);
        bd.span_hi[k][j] = int32_t(hi_s);
        most = std::max(most, int(hi_s - lo_s + 1));
      }
      bd.ext[k] = most + pmax;
      nspan = std::max(nspan, most);
    }
    bd.nspan = nspan;
    bd.tstride = mfa::table_stride(pmax);
    const int64_t box = int64_t(bd.ext[0]) * bd.ext[1] * bd.ext[2];
    const int64_t lds = box > mfa::kEvalBinMaxLds
                            ? int64_t(mfa::kEvalBinMaxLds) + 1
                            : int64_t(mfa::eval_bin_lds_bytes(nspan, bd.tstride, int(box)));
    dm.bin_lds_bytes = (!rational && lds <= mfa::kEvalBinMaxLds) ? int32_t(lds) : 0;
  }

  const int64_t id = ctx->next_id++;
  ctx->models.emplace(id, dm);
  ctx->used += dm.bytes;
  *model_out = id;
  return MFA_OK;
}

mfa_status mfa_model_free(mfa_ctx* ctx, int64_t model) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  if (it->second.batch_refs > 0) return fail(MFA_ERR_INVALID, "model is used by a live batch");
  DeviceGuard g(ctx->device);
  const hipError_t e = hipDeviceSynchronize();
  (void)hipFree(it->second.mem);
  ctx->used -= it->second.bytes;
  ctx->models.erase(it);
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("hipDeviceSynchronize", e));
  return MFA_OK;
}

mfa_status mfa_model_bytes(mfa_ctx* ctx, int64_t model, int64_t* bytes_out) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  if (bytes_out == nullptr) return fail(MFA_ERR_INVALID, "null bytes_out");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  *bytes_out = it->second.bytes;
  return MFA_OK;
}

}  // extern "C"

namespace {

// Host checks of one render request beyond validate_render: the output
// buffer and the number of samples per ray.
mfa_status check_request(const DeviceModel& dm, const mfa_camera* cam, const mfa_tf* tf,
                         const mfa_render_params* prm, const float* rgba_dev) {
  std::string msg;
  const mfa_status st = validate_render(cam, tf, prm, msg);
  if (st != MFA_OK) return fail(st, msg);
  if (rgba_dev == nullptr) return fail(MFA_ERR_INVALID, "null rgba_dev");
  double diag2 = 0.0;
  for (int k = 0; k < 3; ++k) diag2 += (dm.hi[k] - dm.lo[k]) * (dm.hi[k] - dm.lo[k]);
  if (std::sqrt(diag2) / prm->step > double(mfa::kMaxSamplesPerRay))
    return fail(MFA_ERR_INVALID, "step too small: more than 65536 samples per ray");
  return MFA_OK;
}

// Kernel record of one validated request (camera frame, transfer function
// at tf_dev, shading, LDS plan; curv, batch: planned for the occupancy of
// the curvature variants or of the batch kernel).  The tile-plan scratch pointers are left for the caller;
// ntiles receives the request's super-tiles (0 when the request uses the
// global-memory kernel).
void build_render_args(const DeviceModel& dm, const mfa_camera* cam, const mfa_tf* tf,
                       const mfa_render_params* prm, float* rgba_dev, int64_t* samples_dev,
                       float4* tf_dev, mfa::RenderArgsDev& a, bool curv = false,
                       bool batch = false) {
  Frame fr;
  camera_frame(cam, fr);
  a = mfa::RenderArgsDev{};
  a.m = dm.md;
  a.kind = cam->kind;
  a.width = cam->width;
  a.height = cam->height;
  a.ntf = tf->n;
  mfa::CamParams& c = a.cam;
  c.kind = cam->kind;
  c.width = cam->width;
  c.height = cam->height;
  for (int k = 0; k < 3; ++k) {
    c.eye[k] = cam->eye[k];
    c.F[k] = fr.F[k];
    c.R[k] = fr.R[k];
    c.V[k] = fr.V[k];
    c.lo[k] = dm.lo[k];
    c.hi[k] = dm.hi[k];
    c.inv_ext[k] = dm.md.ax[k].inv_ext;
  }
  if (cam->kind == MFA_CAMERA_ORTHO) {
    c.cam0 = cam->ortho_half_w;
    c.cam1 = cam->ortho_half_h;
  } else {
    const double half = cam->fov_y_deg * (M_PI / 180.0) * 0.5;
    c.cam0 = std::tan(half);
    c.cam1 = double(cam->width) / double(cam->height);
  }
  c.step = prm->step;
  a.tf = tf_dev;
  a.tf_lo = float(tf->v_lo);
  a.tf_scale = float(1.0 / (tf->v_hi - tf->v_lo));
  a.ert = float(prm->ert_alpha);
  a.shading = prm->shading;
  a.shininess = prm->shininess;
  a.ka = float(prm->ka);
  a.kd = float(prm->kd);
  a.ks = float(prm->ks);
  if (prm->headlight) {
    for (int k = 0; k < 3; ++k) a.light[k] = float(-fr.F[k]);
  } else {
    const double* l = prm->light_dir;
    const double ll = std::sqrt(l[0] * l[0] + l[1] * l[1] + l[2] * l[2]);
    for (int k = 0; k < 3; ++k) a.light[k] = float(l[k] / ll);
  }
  a.out = rgba_dev;
  a.samples = reinterpret_cast<unsigned long long*>(samples_dev);
  a.fast = dm.md.uniform && dm.md.ax[0].p >= 2 && dm.md.ax[1].p >= 2 && dm.md.ax[2].p >= 2;
  // curvature renders use four lanes per ray (the only variant compiled)
  a.lpr = curv ? mfa::kLanesPerRay : dm.lanes_per_ray;
  a.eq = dm.md.ax[0].p == dm.md.pmax && dm.md.ax[1].p == dm.md.pmax && dm.md.ax[2].p == dm.md.pmax;
  plan_bricks(dm, tf->n, prm->step, curv, batch, a);
  if (dm.md.rational) {
    // the brick kernels are non-rational: rational models use the global kernel
    a.lds_bytes = 0;
    a.spr = 0;
    a.brick_cap = 0;
  }
  a.tile_w = mfa::tile_w_of(a.lpr);
  a.tile_h = mfa::tile_h_of(a.lpr);
  a.ntiles = 0;
  a.nslots = 0;
  if (a.lds_bytes > 0) {
    const int nsx = (cam->width + 2 * a.tile_w - 1) / (2 * a.tile_w);
    const int nsy = (cam->height + 2 * a.tile_h - 1) / (2 * a.tile_h);
    a.nsx = nsx;
    a.ntiles = int32_t(int64_t(nsx) * nsy);
    const int R = std::max(1, std::min(mfa::kMaxRegion, int(std::sqrt(a.ntiles / 64.0))));
    a.region = R;
    // super-tiles per XCD group (regions dealt as in the device's xcd_group)
    int64_t group[mfa::kXcdGroups] = {};
    for (int by = 0; by * R < nsy; ++by)
      for (int bx = 0; bx * R < nsx; ++bx) {
        const int w = std::min(R, nsx - bx * R);
        const int h = std::min(R, nsy - by * R);
        group[(bx + 3 * by) & (mfa::kXcdGroups - 1)] += int64_t(w) * h;
      }
    int64_t largest = 0;
    for (int64_t g : group) largest = std::max(largest, g);
    a.nslots = int32_t(largest * mfa::kXcdGroups);
  }
}

// Enqueue a prepared batch on a stream: per kernel class the planning
// passes and one ray-casting launch; requests on the global-memory kernel
// one by one.
hipError_t launch_batch(const RenderBatch& b, hipStream_t st) {
  for (const auto& c : b.classes) {
    const hipError_t e = mfa::launch_render_batch(c.second, c.first, st);
    if (e != hipSuccess) return e;
  }
  for (const auto& a : b.single) {
    const hipError_t e = mfa::launch_render(a, st, mfa::KernelEvents{});
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Two-phase construction of a render batch: prepare() checks the requests
// and lays out one device block (transfer-function tables, then per kernel
// class the request records, tile prefix sums and planning scratch);
// materialize() writes the block's host image for a given device address
// and the launch description.  The requests' host structures are read by
// prepare() only.
class BatchBuilder {
 public:
  mfa_status prepare(const DeviceModel* const* dms, const mfa_render_request* reqs, int32_t n) {
    std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
    for (int32_t i = 0; i < n; ++i) {
      const mfa_render_request& r = reqs[i];
      const mfa_status st = check_request(*dms[i], r.camera, r.tf, r.params, r.rgba_dev);
      if (st != MFA_OK) return fail(st, "request " + std::to_string(i) + ": " + g_last_error);
      const uintptr_t o = reinterpret_cast<uintptr_t>(r.rgba_dev);
      ranges.emplace_back(o, o + size_t(r.camera->width) * size_t(r.camera->height) * 16);
      if (r.samples_dev != nullptr) {
        const uintptr_t c = reinterpret_cast<uintptr_t>(r.samples_dev);
        ranges.emplace_back(c, c + sizeof(int64_t));
      }
    }
    std::sort(ranges.begin(), ranges.end());
    for (size_t i = 1; i < ranges.size(); ++i)
      if (ranges[i].first < ranges[i - 1].second)
        return fail(MFA_ERR_INVALID, "output buffers of a batch overlap");
    args_.resize(n);
    tf_off_.resize(n);
    tables_.resize(n);
    size_t off = 0;
    for (int32_t i = 0; i < n; ++i) {
      const mfa_render_request& r = reqs[i];
      build_render_args(*dms[i], r.camera, r.tf, r.params, r.rgba_dev, r.samples_dev, nullptr,
                        args_[i], false, true);
      tables_[i].assign(r.tf->rgba, r.tf->rgba + size_t(r.tf->n) * 4);
      tf_off_[i] = off;
      off = align256(off + size_t(r.tf->n) * 16);
    }
    for (int32_t i = 0; i < n; ++i) {
      const mfa::RenderArgsDev& a = args_[i];
      if (a.ntiles == 0) {
        single_.push_back(i);
        continue;
      }
      const mfa::BatchKey k{a.m.pmax, a.m.store, a.shading, a.fast, a.eq, a.lpr, 0};
      Group* gp = nullptr;
      for (auto& g : groups_)
        if (g.key.pmax == k.pmax && g.key.store == k.store && g.key.shading == k.shading &&
            g.key.fast == k.fast && g.key.eq == k.eq && g.key.lpr == k.lpr)
          gp = &g;
      if (gp == nullptr) {
        groups_.push_back(Group{k, {}, 0, 0, 0, 0, 0, 0});
        gp = &groups_.back();
      }
      gp->reqs.push_back(i);
      gp->key.lds_bytes = std::max(gp->key.lds_bytes, a.lds_bytes);
      gp->ntiles += a.ntiles;
    }
    for (auto& g : groups_) {
      if (g.ntiles > int64_t(INT32_MAX)) return fail(MFA_ERR_INVALID, "batch has too many tiles");
      g.off_args = off;
      off = align256(off + sizeof(mfa::RenderArgsDev) * g.reqs.size());
      g.off_base = off;
      off = align256(off + sizeof(int32_t) * (g.reqs.size() + 1));
      g.off_cost = off;
      off = align256(off + sizeof(int32_t) * size_t(g.ntiles));
      g.off_order = off;
      off = align256(off + sizeof(int32_t) * size_t(g.ntiles));
      g.off_hist = off;
      off = align256(off + 4096);
    }
    bytes_ = off;
    return MFA_OK;
  }

  size_t bytes() const { return bytes_; }

  // host: bytes() zeroed bytes, copied to dev before the batch runs
  void materialize(char* dev, unsigned char* host, RenderBatch& b) {
    for (size_t i = 0; i < args_.size(); ++i) {
      std::memcpy(host + tf_off_[i], tables_[i].data(), tables_[i].size() * sizeof(float));
      args_[i].tf = reinterpret_cast<const float4*>(dev + tf_off_[i]);
    }
    b.classes.clear();
    b.single.clear();
    for (auto& gr : groups_) {
      mfa::BatchDev bd{};
      bd.args = reinterpret_cast<const mfa::RenderArgsDev*>(dev + gr.off_args);
      bd.tile_base = reinterpret_cast<const int32_t*>(dev + gr.off_base);
      bd.nreq = int32_t(gr.reqs.size());
      bd.ntiles = int32_t(gr.ntiles);
      bd.tile_cost = reinterpret_cast<int32_t*>(dev + gr.off_cost);
      bd.tile_order = reinterpret_cast<int32_t*>(dev + gr.off_order);
      bd.tile_hist = reinterpret_cast<unsigned*>(dev + gr.off_hist);
      auto* ha = reinterpret_cast<mfa::RenderArgsDev*>(host + gr.off_args);
      auto* hb = reinterpret_cast<int32_t*>(host + gr.off_base);
      int32_t acc = 0;
      for (size_t j = 0; j < gr.reqs.size(); ++j) {
        ha[j] = args_[gr.reqs[j]];
        hb[j] = acc;
        acc += ha[j].ntiles;
      }
      hb[gr.reqs.size()] = acc;
      b.classes.emplace_back(gr.key, bd);
    }
    for (int32_t i : single_) b.single.push_back(args_[i]);
  }

 private:
  struct Group {
    mfa::BatchKey key;
    std::vector<int32_t> reqs;
    size_t off_args, off_base, off_cost, off_order, off_hist;
    int64_t ntiles;
  };
  std::vector<mfa::RenderArgsDev> args_;
  std::vector<size_t> tf_off_;
  std::vector<std::vector<float>> tables_;
  std::vector<Group> groups_;
  std::vector<int32_t> single_;
  size_t bytes_ = 0;
};

}  // namespace

namespace {

// Launch one frame; while kernel timing is on, with a pair of HIP events
// around the ray-casting kernel (at most kMaxTimedLaunches per record).
mfa_status launch_timed(mfa_ctx* ctx, mfa::RenderArgsDev& a, PlanScratch* ps, void* stream) {
  if (ps != nullptr) plan_counters(*ps, a);
  mfa::KernelEvents ev;
  if (ctx->timing && ctx->timed < kMaxTimedLaunches) {
    if (ctx->timed == ctx->events.size()) {
      mfa::KernelEvents fresh;
      hipError_t e = hipEventCreate(&fresh.begin);
      if (e == hipSuccess) {
        e = hipEventCreate(&fresh.end);
        if (e != hipSuccess) (void)hipEventDestroy(fresh.begin);
      }
      if (e != hipSuccess) {
        plan_unready(ctx, stream);
        return fail(MFA_ERR_DEVICE, hip_msg("hipEventCreate", e));
      }
      ctx->events.push_back(fresh);
    }
    ev = ctx->events[ctx->timed];
  }
  const hipError_t e = mfa::launch_render(a, static_cast<hipStream_t>(stream), ev);
  if (e != hipSuccess) {
    plan_unready(ctx, stream);
    return fail(MFA_ERR_DEVICE, hip_msg("render launch", e));
  }
  if (ev.begin != nullptr) ctx->timed += 1;
  return MFA_OK;
}

}  // namespace

extern "C" {

mfa_status mfa_render(mfa_ctx* ctx, int64_t model, const mfa_camera* cam, const mfa_tf* tf,
                      const mfa_render_params* prm, float* rgba_dev, int64_t* samples_dev,
                      void* stream) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  const DeviceModel& dm = it->second;
  mfa_status st = check_request(dm, cam, tf, prm, rgba_dev);
  if (st != MFA_OK) return st;

  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  float4* tf_dev = nullptr;
  st = tf_device(ctx, tf, &tf_dev);
  if (st != MFA_OK) return st;

  mfa::RenderArgsDev a;
  build_render_args(dm, cam, tf, prm, rgba_dev, samples_dev, tf_dev, a);
  PlanScratch* ps = nullptr;
  if (a.ntiles > 0) {
    st = attach_plan(ctx, stream, a.nslots, &a, 1, &ps);
    if (st != MFA_OK) return st;
  }
  return launch_timed(ctx, a, ps, stream);
}

mfa_status mfa_render_noalloc(mfa_ctx* ctx, int64_t model, const mfa_camera* cam,
                              const mfa_tf* tf, const mfa_render_params* prm, float* rgba_dev,
                              int64_t* samples_dev, void* stream) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  const DeviceModel& dm = it->second;
  mfa_status st = check_request(dm, cam, tf, prm, rgba_dev);
  if (st != MFA_OK) return st;
  if (ctx->scratch == nullptr) return fail(MFA_ERR_DEVICE, "no scratch address for this device");
  if (size_t(tf->n) * sizeof(float4) > mfa::kNoAllocTfBytes)
    return fail(MFA_ERR_INVALID, "transfer function larger than the fixed scratch holds");

  char* base = static_cast<char*>(ctx->scratch);
  float4* tf_dev = reinterpret_cast<float4*>(base + mfa::kNoAllocTfOff);
  mfa::RenderArgsDev a;
  build_render_args(dm, cam, tf, prm, rgba_dev, samples_dev, tf_dev, a);
  if (int64_t(a.nslots) > mfa::kNoAllocMaxSlots)
    return fail(MFA_ERR_INVALID, "image too large for the fixed scratch: " +
                                     std::to_string(a.nslots) + " launch slots, at most " +
                                     std::to_string(mfa::kNoAllocMaxSlots));

  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(tf_dev, tf->rgba, size_t(tf->n) * sizeof(float4),
                                hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("transfer function copy", e));
  if (a.ntiles > 0) {
    // the tile sort's counters start at zero: cleared by a fill kernel on
    // every call, since the last call on this GPU left its counts there
    unsigned* counters = reinterpret_cast<unsigned*>(base + mfa::kNoAllocCountersOff);
    e = mfa::launch_plan_init(counters, s);
    if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("scratch clear", e));
    a.tile_cost = reinterpret_cast<int32_t*>(base + mfa::kNoAllocSlotsOff);
    a.tile_order = a.tile_cost + mfa::kNoAllocMaxSlots;
    a.tile_hist = counters;
    a.tile_clear = counters + 2 * mfa::kPlanHistWords;
  }
  e = mfa::launch_render(a, s, mfa::KernelEvents{});
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("render launch", e));
  return MFA_OK;
}

mfa_status mfa_render_curvature(mfa_ctx* ctx, int64_t model, const mfa_camera* cam,
                                const mfa_tf* tf, const mfa_curvature_tf* ctf,
                                const mfa_render_params* prm, float* rgba_dev,
                                int64_t* samples_dev, void* stream) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  const DeviceModel& dm = it->second;
  mfa_status st = check_request(dm, cam, tf, prm, rgba_dev);
  if (st != MFA_OK) return st;
  if (ctf == nullptr || ctf->rgba == nullptr || ctf->m < 2 || ctf->m > MFA_MAX_CURV_TF)
    return fail(MFA_ERR_INVALID, "curvature table needs 2..64 entries per axis");
  if (!(std::isfinite(ctf->k_lo) && std::isfinite(ctf->k_hi) && ctf->k_lo < ctf->k_hi))
    return fail(MFA_ERR_INVALID, "curvature range needs finite k_lo < k_hi");
  const int nent = ctf->m * ctf->m;
  for (int i = 0; i < 4 * nent; ++i) {
    if (!std::isfinite(ctf->rgba[i]) ||
        (i % 4 == 3 && !(ctf->rgba[i] >= 0.0f && ctf->rgba[i] <= 1.0f)))
      return fail(MFA_ERR_INVALID, "curvature table entries must be finite, opacities in [0, 1]");
  }
  if (dm.md.rational) return fail(MFA_ERR_MODEL, "curvature rendering needs a non-rational model");

  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  // room for both tables first: a full cache is released on insertion
  if (ctx->n_tf + 2 > kMaxCachedTF) {
    const hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("hipDeviceSynchronize", e));
    ctx->free_tfs();
  }
  float4* tf_dev = nullptr;
  st = tf_device(ctx, tf, &tf_dev);
  if (st != MFA_OK) return st;
  mfa_tf flat{};
  flat.n = nent;
  flat.rgba = ctf->rgba;
  flat.v_lo = ctf->k_lo;
  flat.v_hi = ctf->k_hi;
  float4* ctf_dev = nullptr;
  st = tf_device(ctx, &flat, &ctf_dev);
  if (st != MFA_OK) return st;

  // the brick ray caster with second derivatives (the global-memory kernel
  // when the transfer function leaves too little LDS for bricks)
  mfa::RenderArgsDev a;
  build_render_args(dm, cam, tf, prm, rgba_dev, samples_dev, tf_dev, a, true);
  a.ctf = ctf_dev;
  a.ctf_m = ctf->m;
  a.ctf_lo = float(ctf->k_lo);
  a.ctf_scale = float(1.0 / (ctf->k_hi - ctf->k_lo));
  PlanScratch* ps = nullptr;
  if (a.ntiles > 0) {
    st = attach_plan(ctx, stream, a.nslots, &a, 1, &ps);
    if (st != MFA_OK) return st;
  }
  return launch_timed(ctx, a, ps, stream);
}

mfa_status mfa_measure_fma_peak(mfa_ctx* ctx, double* tflops) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  if (tflops == nullptr) return fail(MFA_ERR_INVALID, "null tflops");
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  int cus = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
  if (e != hipSuccess || cus <= 0) return fail(MFA_ERR_DEVICE, hip_msg("CU count", e));
  const int blocks = 16 * cus;   // 16 workgroups of 4 waves per CU
  const int iters = 20000;
  float* out = nullptr;
  e = hipMalloc(reinterpret_cast<void**>(&out), sizeof(float) * size_t(blocks));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MFA_ERR_NOMEM, hip_msg("hipMalloc (FMA probe)", e));
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  float ms = 0.0f;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e == hipSuccess) e = mfa::launch_fma_peak(out, blocks, 100, nullptr);   // warm-up
  if (e == hipSuccess) e = hipEventRecord(t0, nullptr);
  if (e == hipSuccess) e = mfa::launch_fma_peak(out, blocks, iters, nullptr);
  if (e == hipSuccess) e = hipEventRecord(t1, nullptr);
  if (e == hipSuccess) e = hipEventSynchronize(t1);
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, t0, t1);
  if (t0 != nullptr) (void)hipEventDestroy(t0);
  if (t1 != nullptr) (void)hipEventDestroy(t1);
  (void)hipFree(out);
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("FMA probe", e));
  const double flops = double(blocks) * 256.0 * double(iters) * 8.0 * 2.0;
  *tflops = flops / (double(ms) * 1e-3) / 1e12;
  return MFA_OK;
}

mfa_status mfa_kernel_timing(mfa_ctx* ctx, int32_t enable) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  ctx->timing = enable != 0;
  ctx->timed = 0;
  return MFA_OK;
}

mfa_status mfa_kernel_times(mfa_ctx* ctx, float* ms_host, int64_t cap, int64_t* count) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  if (count == nullptr || cap < 0 || (cap > 0 && ms_host == nullptr))
    return fail(MFA_ERR_INVALID, "null count, negative cap or null ms_host");
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  const size_t n = ctx->timed;
  for (size_t i = 0; i < n; ++i) {
    hipError_t e = hipEventSynchronize(ctx->events[i].end);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, ctx->events[i].begin, ctx->events[i].end);
    if (e != hipSuccess) {
      ctx->timed = 0;
      return fail(MFA_ERR_DEVICE, hip_msg("kernel timing events", e));
    }
    if (int64_t(i) < cap) ms_host[i] = ms;
  }
  *count = int64_t(n);
  ctx->timed = 0;
  return MFA_OK;
}

mfa_status mfa_autotune(mfa_ctx* ctx, int64_t model, const mfa_camera* cam, const mfa_tf* tf,
                        const mfa_render_params* prm, float* rgba_dev, int32_t repeats,
                        void* stream, mfa_tune_result* out) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  if (repeats < 1 || repeats > 1000) return fail(MFA_ERR_INVALID, "repeats must be in [1, 1000]");
  DeviceModel& dm = it->second;
  mfa_status st = check_request(dm, cam, tf, prm, rgba_dev);
  if (st != MFA_OK) return st;
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  float4* tf_dev = nullptr;
  st = tf_device(ctx, tf, &tf_dev);
  if (st != MFA_OK) return st;
  const hipStream_t hs = static_cast<hipStream_t>(stream);
  // one launch record per candidate; launches of all candidates are
  // interleaved (round robin) and enqueued back to back, with events around
  // each ray-casting kernel, and the stream is synchronised once
  // candidates: every lanes-per-ray count with every round length
  constexpr int kSpans = int(sizeof(kTuneRoundSpans) / sizeof(kTuneRoundSpans[0]));
  constexpr int kLanes = int(sizeof(kTuneLanes) / sizeof(kTuneLanes[0]));
  constexpr int kCand = kSpans * kLanes;
  const double saved = dm.round_spans;
  const int32_t saved_lanes = dm.lanes_per_ray;
  std::vector<mfa::RenderArgsDev> args(kCand);
  int64_t slots = 0;
  for (int c = 0; c < kCand; ++c) {
    dm.round_spans = kTuneRoundSpans[c % kSpans];
    dm.lanes_per_ray = kTuneLanes[c / kSpans];
    build_render_args(dm, cam, tf, prm, rgba_dev, nullptr, tf_dev, args[c]);
    slots = std::max<int64_t>(slots, args[c].nslots);
  }
  dm.round_spans = saved;
  dm.lanes_per_ray = saved_lanes;
  PlanScratch* ps = nullptr;
  if (args[0].ntiles > 0) {
    st = attach_plan(ctx, stream, slots, args.data(), kCand, &ps);
    if (st != MFA_OK) return st;
  }
  const int total = kCand * (repeats + 1);
  std::vector<mfa::KernelEvents> evs(total);
  hipError_t e = hipSuccess;
  int made = 0;
  for (; made < total && e == hipSuccess; ++made) {
    e = hipEventCreate(&evs[made].begin);
    if (e == hipSuccess) {
      e = hipEventCreate(&evs[made].end);
      if (e != hipSuccess) (void)hipEventDestroy(evs[made].begin);
    }
  }
  if (e != hipSuccess) --made;
  for (int r = 0, k = 0; r <= repeats && e == hipSuccess; ++r)   // round 0: warm-up
    for (int c = 0; c < kCand && e == hipSuccess; ++c, ++k) {
      if (ps != nullptr) plan_counters(*ps, args[c]);
      e = mfa::launch_render(args[c], hs, evs[k]);
    }
  if (e != hipSuccess) plan_unready(ctx, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(hs);
  double best = saved, best_ms = 1e30, default_ms = 0.0;
  int32_t best_lanes = saved_lanes;
  for (int c = 0; c < kCand && e == hipSuccess; ++c) {
    std::vector<float> ms;
    for (int r = 1; r <= repeats && e == hipSuccess; ++r) {
      float t = 0.0f;
      e = hipEventElapsedTime(&t, evs[r * kCand + c].begin, evs[r * kCand + c].end);
      ms.push_back(t);
    }
    if (e != hipSuccess) break;
    std::sort(ms.begin(), ms.end());
    const double med = ms[ms.size() / 2];
    const double spans = kTuneRoundSpans[c % kSpans];
    const int32_t lanes = kTuneLanes[c / kSpans];
    if (spans == 3.0 && lanes == mfa::kLanesPerRay) default_ms = med;
    if (med < best_ms) {
      best_ms = med;
      best = spans;
      best_lanes = lanes;
    }
  }
  for (int i = 0; i < made; ++i) {
    (void)hipEventDestroy(evs[i].begin);
    (void)hipEventDestroy(evs[i].end);
  }
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("autotune launch", e));
  const int32_t tried = kCand;
  dm.round_spans = best;
  dm.lanes_per_ray = best_lanes;
  if (out != nullptr) {
    out->round_spans = float(best);
    out->lanes_per_ray = best_lanes;
    out->candidates = tried;
    out->best_ms = float(best_ms);
    out->default_ms = float(default_ms);
  }
  return MFA_OK;
}

mfa_status mfa_model_set_tuning(mfa_ctx* ctx, int64_t model, float round_spans,
                                int32_t lanes_per_ray) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  if (!(round_spans >= 0.5f && round_spans <= 16.0f))
    return fail(MFA_ERR_INVALID, "round_spans must be in [0.5, 16]");
  if (lanes_per_ray != 1 && lanes_per_ray != 2 && lanes_per_ray != 4)
    return fail(MFA_ERR_INVALID, "lanes_per_ray must be 1, 2 or 4");
  it->second.round_spans = round_spans;
  it->second.lanes_per_ray = lanes_per_ray;
  return MFA_OK;
}

mfa_status mfa_batch_create(mfa_ctx* ctx, const mfa_render_request* reqs, int32_t n,
                            int64_t* batch_out) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  if (batch_out == nullptr || reqs == nullptr) return fail(MFA_ERR_INVALID, "null argument");
  if (n < 1 || n > kMaxBatch) return fail(MFA_ERR_INVALID, "batch size must be in [1, 65536]");
  std::vector<const DeviceModel*> dms(n);
  for (int32_t i = 0; i < n; ++i) {
    auto it = ctx->models.find(reqs[i].model);
    if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle in batch");
    dms[i] = &it->second;
  }
  BatchBuilder bb;
  mfa_status st = bb.prepare(dms.data(), reqs, n);
  if (st != MFA_OK) return st;
  const size_t bytes = bb.bytes();
  if (ctx->budget > 0 && ctx->used + int64_t(bytes) > ctx->budget)
    return fail(MFA_ERR_NOMEM, "batch exceeds the context's memory budget");
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(MFA_ERR_NOMEM, hip_msg("hipMalloc (batch)", e));
  }
  std::vector<unsigned char> host(bytes, 0);
  RenderBatch b;
  bb.materialize(static_cast<char*>(mem), host.data(), b);
  b.mem = mem;
  b.bytes = int64_t(bytes);
  e = hipMemcpy(mem, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return fail(MFA_ERR_DEVICE, hip_msg("hipMemcpy (batch)", e));
  }
  for (int32_t i = 0; i < n; ++i) {
    ctx->models[reqs[i].model].batch_refs += 1;
    b.models.push_back(reqs[i].model);
  }
  ctx->used += b.bytes;
  const int64_t id = ctx->next_id++;
  ctx->batches.emplace(id, std::move(b));
  *batch_out = id;
  return MFA_OK;
}

mfa_status mfa_batch_render(mfa_ctx* ctx, int64_t batch, void* stream) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->batches.find(batch);
  if (it == ctx->batches.end()) return fail(MFA_ERR_HANDLE, "unknown batch handle");
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  const hipError_t e = launch_batch(it->second, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("batch launch", e));
  return MFA_OK;
}

mfa_status mfa_batch_free(mfa_ctx* ctx, int64_t batch) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->batches.find(batch);
  if (it == ctx->batches.end()) return fail(MFA_ERR_HANDLE, "unknown batch handle");
  DeviceGuard g(ctx->device);
  const hipError_t e = hipDeviceSynchronize();
  (void)hipFree(it->second.mem);
  ctx->used -= it->second.bytes;
  for (int64_t m : it->second.models) {
    auto mi = ctx->models.find(m);
    if (mi != ctx->models.end()) mi->second.batch_refs -= 1;
  }
  ctx->batches.erase(it);
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("hipDeviceSynchronize", e));
  return MFA_OK;
}

}  // extern "C"

namespace {

// Point queries: value, optional world gradient, optional world Hessian.
mfa_status eval_common(mfa_ctx* ctx, int64_t model, int64_t n, const double* xyz_dev,
                       float* value_dev, float* grad_dev, float* hess_dev, void* stream) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  auto it = ctx->models.find(model);
  if (it == ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  if (n < 0 || n > kMaxEvalPoints) return fail(MFA_ERR_INVALID, "point count out of range");
  if (n == 0) return MFA_OK;
  if (xyz_dev == nullptr || value_dev == nullptr)
    return fail(MFA_ERR_INVALID, "null point or value buffer");
  const DeviceModel& dm = it->second;
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  mfa::EvalArgsDev a{};
  a.m = dm.md;
  for (int k = 0; k < 3; ++k) {
    a.lo[k] = dm.lo[k];
    a.hi[k] = dm.hi[k];
  }
  a.xyz = xyz_dev;
  a.value = value_dev;
  a.grad = grad_dev;
  a.hess = hess_dev;
  a.n = n;
  a.order = nullptr;
  a.use_order = nullptr;
  const double score = std::sqrt(double(dm.md.ctrl_bytes) + double(dm.md.wctrl_bytes)) *
                       std::pow(double(dm.md.pmax + 1), 3.0);
  if (n >= kEvalOrderMin && n <= int64_t(INT32_MAX) && score >= kEvalOrderScore) {
    mfa::EvalOrderDev o{};
    // binned evaluation from LDS where the model's slabs fit: always
    // sorted; otherwise gathers, in bin order unless the probe finds the
    // points already local
    const bool binned = dm.bin_lds_bytes > 0;
    const mfa_status st = attach_eval(ctx, stream, n, o);
    if (st == MFA_ERR_NOMEM) {
      // the order is an optimisation: without its scratch, evaluate the
      // points as given
      g_last_error.clear();
      const hipError_t e = mfa::launch_eval(a, static_cast<hipStream_t>(stream));
      if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("eval launch", e));
      return MFA_OK;
    }
    if (st != MFA_OK) return st;
    o.xyz = xyz_dev;
    o.n = n;
    for (int k = 0; k < 3; ++k) {
      o.lo[k] = dm.md.ax[k].lo;
      o.inv_ext[k] = dm.md.ax[k].inv_ext;
    }
    o.force = binned ? 1 : 0;
    o.bins = binned ? 1 : 0;
    o.groups = int32_t((n + mfa::kEvalSortChunk - 1) / mfa::kEvalSortChunk);
    const hipError_t eo = mfa::launch_eval_order(o, static_cast<hipStream_t>(stream));
    if (eo != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("point order launch", eo));
    if (binned) {
      mfa::EvalBinDev bd = dm.bins;
      bd.order = o.idx[mfa::kEvalPasses % 2];
      bd.bin_start = o.bin_start;
      bd.item_base = o.item_base;
      bd.flags = o.flags;
      const hipError_t eb =
          mfa::launch_eval_bins(a, bd, dm.bin_lds_bytes, static_cast<hipStream_t>(stream));
      if (eb != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("binned eval launch", eb));
      return MFA_OK;
    }
    a.order = o.idx[mfa::kEvalPasses % 2];
    a.use_order = o.flags + 1;
  }
  const hipError_t e = mfa::launch_eval(a, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("eval launch", e));
  return MFA_OK;
}

}  // namespace

extern "C" {

mfa_status mfa_eval_points(mfa_ctx* ctx, int64_t model, int64_t n, const double* xyz_dev,
                           float* value_dev, float* grad_dev, void* stream) {
  return eval_common(ctx, model, n, xyz_dev, value_dev, grad_dev, nullptr, stream);
}

mfa_status mfa_eval_hessian(mfa_ctx* ctx, int64_t model, int64_t n, const double* xyz_dev,
                            float* value_dev, float* grad_dev, float* hess_dev, void* stream) {
  g_last_error.clear();
  if (ctx != nullptr && hess_dev == nullptr && n > 0)
    return fail(MFA_ERR_INVALID, "null Hessian buffer");
  if (ctx != nullptr) {
    auto it = ctx->models.find(model);
    if (it != ctx->models.end() && it->second.md.rational)
      return fail(MFA_ERR_MODEL, "Hessian queries need a non-rational model");
  }
  return eval_common(ctx, model, n, xyz_dev, value_dev, grad_dev, hess_dev, stream);
}

}  // extern "C"

// --------------------------------------------------------------------------
// serving: continuous batching of render requests
// --------------------------------------------------------------------------

namespace {

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// A submitted request with private copies of everything it points to.
struct Pending {
  int64_t ticket = 0;
  int64_t model = 0;
  DeviceModel dm;              // copy of the model record (device pointers)
  mfa_camera cam{};
  mfa_render_params prm{};
  std::vector<float> table;
  mfa_tf tf{};
  float* rgba = nullptr;
  int64_t* samples = nullptr;
  int64_t footprint = 0;       // output bytes plus an estimate of its share of a batch block
  int64_t submit_ns = 0;
  bool deferred = false;       // held back by the byte budget while a slot was free
};

struct TicketState {
  mfa_request_info info{};
  bool finished = false;
};

// One launch slot: a stream, its completion event, a reusable device block
// and pinned staging for the block's host image.  A slot is reused only
// after its event has completed.
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  unsigned char* staging = nullptr;
  size_t staging_bytes = 0;
  bool busy = false;
  int64_t bytes = 0;            // footprint of the requests in flight
  std::vector<Pending> reqs;
};

}  // namespace

struct mfa_server {
  mfa_ctx* ctx = nullptr;
  mfa_server_config cfg{};
  std::mutex mu;
  std::condition_variable work_cv;   // submitters -> worker
  std::condition_variable done_cv;   // worker -> waiters
  std::deque<Pending> queue;
  std::unordered_map<int64_t, TicketState> tickets;
  std::vector<Slot> slots;
  int64_t next_ticket = 1;
  int64_t in_flight_bytes = 0;
  bool stop = false;
  std::thread worker;
  std::string worker_error;
};

namespace {

// Grow a slot's device block and pinned staging to `bytes`; the slot is idle.
hipError_t slot_reserve(Slot& sl, size_t bytes) {
  if (sl.arena_bytes < bytes) {
    if (sl.arena != nullptr) (void)hipFree(sl.arena);
    sl.arena = nullptr;
    sl.arena_bytes = 0;
    const size_t want = std::max(bytes, size_t(1) << 20) * 3 / 2;
    const hipError_t e = hipMalloc(&sl.arena, want);
    if (e != hipSuccess) return e;
    sl.arena_bytes = want;
  }
  if (sl.staging_bytes < bytes) {
    if (sl.staging != nullptr) (void)hipHostFree(sl.staging);
    sl.staging = nullptr;
    sl.staging_bytes = 0;
    const size_t want = std::max(bytes, size_t(1) << 20) * 3 / 2;
    const hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&sl.staging), want, 0);
    if (e != hipSuccess) return e;
    sl.staging_bytes = want;
  }
  return hipSuccess;
}

// Finish the requests of a slot (status st), under the server lock.
void slot_retire(mfa_server* sv, Slot& sl, mfa_status st) {
  const int64_t t = now_ns();
  for (auto& r : sl.reqs) {
    auto it = sv->tickets.find(r.ticket);
    if (it != sv->tickets.end()) {
      it->second.info.status = st;
      it->second.info.done_ns = t;
      it->second.finished = true;
    }
    auto mi = sv->ctx->models.find(r.model);
    if (mi != sv->ctx->models.end()) mi->second.batch_refs -= 1;
  }
  sv->in_flight_bytes -= sl.bytes;
  sl.reqs.clear();
  sl.bytes = 0;
  sl.busy = false;
}

// Build the batch of a slot's requests into its block and enqueue it.
// Called without the server lock (the slot's requests are owned by the
// worker until it retires them).
mfa_status slot_launch(Slot& sl) {
  const int32_t n = int32_t(sl.reqs.size());
  std::vector<const DeviceModel*> dms(n);
  std::vector<mfa_render_request> rq(n);
  for (int32_t i = 0; i < n; ++i) {
    Pending& p = sl.reqs[i];
    p.tf.rgba = p.table.data();
    dms[i] = &p.dm;
    rq[i] = mfa_render_request{p.model, &p.cam, &p.tf, &p.prm, p.rgba, p.samples};
  }
  BatchBuilder bb;
  mfa_status st = bb.prepare(dms.data(), rq.data(), n);
  if (st != MFA_OK) return st;
  const size_t bytes = bb.bytes();
  hipError_t e = slot_reserve(sl, bytes);
  if (e != hipSuccess) return fail(MFA_ERR_NOMEM, hip_msg("server block", e));
  std::memset(sl.staging, 0, bytes);
  RenderBatch b;
  bb.materialize(static_cast<char*>(sl.arena), sl.staging, b);
  e = hipMemcpyAsync(sl.arena, sl.staging, bytes, hipMemcpyHostToDevice, sl.stream);
  if (e == hipSuccess) e = launch_batch(b, sl.stream);
  if (e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
  if (e != hipSuccess) return fail(MFA_ERR_DEVICE, hip_msg("server launch", e));
  return MFA_OK;
}

void server_loop(mfa_server* sv) {
  DeviceGuard g(sv->ctx->device);
  std::unique_lock<std::mutex> lk(sv->mu);
  for (;;) {
    bool progress = false;
    // retire finished slots
    for (auto& sl : sv->slots) {
      if (!sl.busy) continue;
      const hipError_t q = hipEventQuery(sl.done);
      if (q == hipErrorNotReady) continue;
      slot_retire(sv, sl, q == hipSuccess ? MFA_OK : MFA_ERR_DEVICE);
      progress = true;
    }
    if (progress) sv->done_cv.notify_all();
    // admit queued requests into a free slot
    Slot* free_slot = nullptr;
    for (auto& sl : sv->slots)
      if (!sl.busy) {
        free_slot = &sl;
        break;
      }
    if (free_slot != nullptr && !sv->queue.empty()) {
      const int64_t budget = sv->cfg.max_bytes;
      while (!sv->queue.empty() && int32_t(free_slot->reqs.size()) < sv->cfg.max_batch) {
        Pending& p = sv->queue.front();
        if (budget > 0 && sv->in_flight_bytes + free_slot->bytes + p.footprint > budget &&
            !(free_slot->reqs.empty() && sv->in_flight_bytes == 0)) {
          p.deferred = true;
          break;
        }
        free_slot->bytes += p.footprint;
        free_slot->reqs.push_back(std::move(p));
        sv->queue.pop_front();
      }
      if (!free_slot->reqs.empty()) {
        free_slot->busy = true;
        sv->in_flight_bytes += free_slot->bytes;
        const int64_t t = now_ns();
        const int32_t nb = int32_t(free_slot->reqs.size());
        for (auto& r : free_slot->reqs) {
          TicketState& ts = sv->tickets[r.ticket];
          ts.info.launch_ns = t;
          ts.info.batch_size = nb;
          ts.info.deferred = r.deferred ? 1 : 0;
        }
        lk.unlock();
        const mfa_status st = slot_launch(*free_slot);
        lk.lock();
        if (st != MFA_OK) {
          (void)hipStreamSynchronize(free_slot->stream);
          slot_retire(sv, *free_slot, st);
          sv->done_cv.notify_all();
        }
        progress = true;
      }
    }
    bool any_busy = false;
    for (auto& sl : sv->slots) any_busy = any_busy || sl.busy;
    if (sv->stop && sv->queue.empty() && !any_busy) break;
    if (!progress) {
      // poll the device while work is in flight, else sleep until a submit
      if (any_busy)
        sv->work_cv.wait_for(lk, std::chrono::microseconds(20));
      else
        sv->work_cv.wait_for(lk, std::chrono::milliseconds(5));
    }
  }
}

}  // namespace

extern "C" {

mfa_status mfa_server_create(mfa_ctx* ctx, const mfa_server_config* cfg, mfa_server** out) {
  g_last_error.clear();
  if (ctx == nullptr) return fail(MFA_ERR_HANDLE, "null context");
  if (out == nullptr) return fail(MFA_ERR_INVALID, "null server_out");
  mfa_server_config c{2, 256, 0};
  if (cfg != nullptr) c = *cfg;
  if (c.streams == 0) c.streams = 2;
  if (c.max_batch == 0) c.max_batch = 256;
  if (c.streams < 1 || c.streams > 8 || c.max_batch < 1 || c.max_batch > kMaxBatch ||
      c.max_bytes < 0)
    return fail(MFA_ERR_INVALID, "server config: streams in [1, 8], max_batch in [1, 65536], "
                                 "max_bytes >= 0");
  DeviceGuard g(ctx->device);
  if (!g.ok()) return fail(MFA_ERR_DEVICE, "hipSetDevice failed");
  auto* sv = new mfa_server;
  sv->ctx = ctx;
  sv->cfg = c;
  sv->slots.resize(c.streams);
  for (auto& sl : sv->slots) {
    hipError_t e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
    if (e != hipSuccess) {
      for (auto& t : sv->slots) {
        if (t.done) (void)hipEventDestroy(t.done);
        if (t.stream) (void)hipStreamDestroy(t.stream);
      }
      delete sv;
      return fail(MFA_ERR_DEVICE, hip_msg("server streams", e));
    }
  }
  sv->worker = std::thread(server_loop, sv);
  *out = sv;
  return MFA_OK;
}

mfa_status mfa_server_submit(mfa_server* sv, const mfa_render_request* req, int64_t* ticket_out) {
  g_last_error.clear();
  if (sv == nullptr) return fail(MFA_ERR_HANDLE, "null server");
  if (req == nullptr || ticket_out == nullptr) return fail(MFA_ERR_INVALID, "null argument");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->stop) return fail(MFA_ERR_INVALID, "server is shutting down");
  auto it = sv->ctx->models.find(req->model);
  if (it == sv->ctx->models.end()) return fail(MFA_ERR_HANDLE, "unknown model handle");
  const mfa_status st = check_request(it->second, req->camera, req->tf, req->params,
                                      req->rgba_dev);
  if (st != MFA_OK) return st;
  Pending p;
  p.model = req->model;
  p.dm = it->second;
  p.cam = *req->camera;
  p.prm = *req->params;
  p.table.assign(req->tf->rgba, req->tf->rgba + size_t(req->tf->n) * 4);
  p.tf = *req->tf;
  p.rgba = req->rgba_dev;
  p.samples = req->samples_dev;
  const int64_t pixels = int64_t(p.cam.width) * p.cam.height;
  p.footprint = pixels * 16 + (pixels / 64 + 1) * 8 + int64_t(p.tf.n) * 16 + 1024;
  if (sv->cfg.max_bytes > 0 && p.footprint > sv->cfg.max_bytes)
    return fail(MFA_ERR_NOMEM, "request exceeds the server's byte budget");
  p.ticket = sv->next_ticket++;
  p.submit_ns = now_ns();
  TicketState& ts = sv->tickets[p.ticket];
  ts.info.status = MFA_OK;
  ts.info.submit_ns = p.submit_ns;
  it->second.batch_refs += 1;
  *ticket_out = p.ticket;
  sv->queue.push_back(std::move(p));
  lk.unlock();
  sv->work_cv.notify_one();
  return MFA_OK;
}

mfa_status mfa_server_wait(mfa_server* sv, int64_t ticket, int64_t timeout_us,
                           mfa_request_info* info) {
  g_last_error.clear();
  if (sv == nullptr) return fail(MFA_ERR_HANDLE, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (sv->tickets.find(ticket) == sv->tickets.end())
    return fail(MFA_ERR_HANDLE, "unknown ticket");
  // finished, or forgotten by another thread's wait on the same ticket
  auto ready = [&] {
    const auto jt = sv->tickets.find(ticket);
    return jt == sv->tickets.end() || jt->second.finished;
  };
  if (timeout_us < 0)
    sv->done_cv.wait(lk, ready);
  else if (!sv->done_cv.wait_for(lk, std::chrono::microseconds(timeout_us), ready))
    return fail(MFA_ERR_TIMEOUT, "request not finished");
  const auto it = sv->tickets.find(ticket);
  if (it == sv->tickets.end()) return fail(MFA_ERR_HANDLE, "ticket already waited for");
  const TicketState ts = it->second;
  sv->tickets.erase(it);
  // other waiters on this ticket see it gone
  sv->done_cv.notify_all();
  if (info != nullptr) *info = ts.info;
  if (ts.info.status != MFA_OK) return fail(ts.info.status, "request failed on the device");
  return MFA_OK;
}

mfa_status mfa_server_destroy(mfa_server* sv) {
  g_last_error.clear();
  if (sv == nullptr) return MFA_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->work_cv.notify_all();
  if (sv->worker.joinable()) sv->worker.join();
  DeviceGuard g(sv->ctx->device);
  for (auto& sl : sv->slots) {
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    if (sl.arena) (void)hipFree(sl.arena);
    if (sl.staging) (void)hipHostFree(sl.staging);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  delete sv;
  return MFA_OK;
}

}  // extern "C"
