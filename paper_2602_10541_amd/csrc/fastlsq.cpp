// libfastlsq: C ABI and host drivers of the MI355X FastLSQ hot path.
//
// Drivers (all FP64 control, kernels in k_*.hip):
//   solve:   Gram (fused assembly + MFMA) -> + mu I -> blocked Cholesky G = U^T U
//            -> beta0 = U^{-1} U^{-T} A^T rhs -> CGLS refinement with FP64 matrix-free
//            products, preconditioned by U (Sections 2.3-2.5: Tikhonov least squares).
//   newton:  warm start (linear part), then per step residual R and Jacobian row
//            coefficient N'(u) (FP64), Gram of J, factor, solve J delta = -R in the
//            Tikhonov sense, Armijo backtracking on ||R|| (Section 2.4, Eq. (4)-(5)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fastlsq.h"
#include "flsq_launch.h"

using namespace flsq;

namespace {

// ------------------------------------------------------------------ device buffers
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t ensure(size_t b) {
    if (b <= bytes && p) return hipSuccess;
    release();
    if (b == 0) b = 256;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    bytes = b;
    return hipSuccess;
  }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

struct Err {
  flsq_status st;
  std::string msg;
};

#define CHECK_HIP(expr)                                                                   \
  do {                                                                                    \
    hipError_t e__ = (expr);                                                              \
    if (e__ != hipSuccess)                                                                \
      return Err{e__ == hipErrorOutOfMemory ? FLSQ_ENOMEM : FLSQ_EHIP,                    \
                 std::string(#expr) + ": " + hipGetErrorString(e__)};                     \
  } while (0)

#define CHECK_ERR(expr)              \
  do {                               \
    Err e__ = (expr);                \
    if (e__.st != FLSQ_OK) return e__; \
  } while (0)

inline Err ok() { return Err{FLSQ_OK, ""}; }
inline Err fail(flsq_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return Err{s, buf};
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------------ problem on the device
struct System {
  int d = 0, n = 0, n_blocks = 0;
  int64_t P = 0;
  double norm = 1.0;
  std::vector<int64_t> row0;          // per block
  std::vector<int64_t> rows;
  std::vector<double> weight;
  std::vector<int> even;              // operator has even-order terms only
  int normalize = 1;
  DevBuf Wt, Wt32, Wrm, bvec, amp, ph, amp32, ph32, Xt, Xt32, Xrm, row_block, rhs_w, chunks, runs, wide, frec;
  int n_chunks = 0, n_runs = 0, n_wide = 0;
  // Gram plan
  int nt = 0, n_wg = 0, max_seg = 0;
  int64_t total_units = 0, units_per_wg = 0;
  DevBuf slot_ptr, slots;

  Geo geo() const {
    Geo g;
    g.d = d;
    g.n = n;
    g.P = P;
    g.n_blocks = n_blocks;
    g.Wt = Wt.as<double>();
    g.Wt32 = Wt32.as<float>();
    g.amp = amp.as<double>();
    g.ph = ph.as<double>();
    g.amp32 = amp32.as<float>();
    g.ph32 = ph32.as<float>();
    g.Xt = Xt.as<double>();
    g.Xrm = Xrm.as<double>();
    g.Xt32 = Xt32.as<float>();
    g.row_block = row_block.as<int32_t>();
    g.frec = frec.as<double>();
    return g;
  }
  PassGeo pass() const {
    PassGeo pg;
    pg.g = geo();
    pg.runs = runs.as<Chunk>();
    pg.n_runs = n_runs;
    pg.wide = wide.as<Chunk>();
    pg.n_wide = n_wide;
    pg.even_mask = 0;
    for (int b = 0; b < n_blocks && b < 64; ++b)
      if (even[b]) pg.even_mask |= 1ull << b;
    pg.norm = norm;
    return pg;
  }
};

}  // namespace

// The shift a factorisation needed, with the fingerprint of its Gram (see factor_with_retries).
struct ShiftMemo {
  bool valid = false;
  int n = 0;
  double mu = 0.0, shift0 = 0.0, boost = 0.0;
  unsigned long long fp = 0;
  double shift = 0.0;
};

struct flsq_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  int n_cu = 256;
  std::string err;
  std::map<std::string, DevBuf> ws;
  System sys;                        // cached system of the last solve_linear / gram / newton call
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t ev_g0 = nullptr, ev_g1 = nullptr;   // around a solve's whole Gram phase
  double last_gram_kernel_ms = 0.0;  // duration of the last fused Gram kernel (HIP events on the stream)
  void* pinned = nullptr;            // pinned host staging for the small per-iteration read-backs
  size_t pinned_bytes = 0;
  void* up = nullptr;                // pinned host staging of small uploads (plans, descriptors, tables)
  size_t up_bytes = 0, up_off = 0;   // bytes in use since the stream was last drained
  flsq_factor* aux_factor = nullptr; // factor and derived system reused by the learnable-bandwidth calls
  System aux;
  unsigned char* scratch = nullptr;  // this device's copy of the static evaluation scratch (no-alloc calls)
  ShiftMemo shift_memo[4];           // recent factorisations that needed a shift retry (one per key)
  int shift_memo_next = 0;           // the entry a new key replaces
};

struct flsq_factor {
  int device = 0;
  System sys;
  // geometry derived for the inverse-problem calls (observation rows, dA/dkappa rows), cached
  System obs, akap;
  const void* obs_key = nullptr;
  int64_t obs_n = -1, akap_rows = -1;
  int akap_dims = -1;
  double akap_weight = 0.0;
  DevBuf Xinv;                       // inverse of the upper Cholesky factor, n x n row-major
  DevBuf Ad, Atd;                    // A (P x n) and A^T (n x P) in MFMA operand order, when kept
  bool dense = false;
  // observation operator R = H (A^T A + mu I)^{-1} A_src^T (n_obs x n_src) and R^T, operand order
  DevBuf R16, Rt16;
  const void* rep_key = nullptr;
  int64_t rep_nobs = -1, rep_nsrc = -1;
  double mu = 0.0;
  double shift = 0.0;
  int max_refine = 0;
  double refine_tol = 0.0;
  bool report_grad = false;
};

// Scratch of the allocation-free evaluation call: one copy per device, held by the process until it
// ends.  Host code never passes `scratch` itself to a kernel or a copy (in host code the name is a
// host-side stand-in, not a device address); it uses the address hipGetSymbolAddress returns for
// the current device, resolved once per device in flsq_create.
static __device__ __align__(256) unsigned char scratch[FLSQ_EVAL_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be current.
hipError_t scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_addr[device] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_addr[device];
  return hipSuccess;
}

DevBuf& wsb(flsq_ctx* c, const std::string& name) { return c->ws[name]; }

template <typename T>
Err ws_get(flsq_ctx* c, const std::string& name, size_t count, T** out) {
  DevBuf& b = wsb(c, name);
  CHECK_HIP(b.ensure(count * sizeof(T)));
  *out = b.as<T>();
  return ok();
}

// Copy `bytes` from the device to host memory through the context's pinned staging buffer and
// wait for the stream (the solvers' stopping decisions read a few scalars per iteration).
Err read_back(flsq_ctx* c, void* host, const void* dev, size_t bytes) {
  if (bytes > c->pinned_bytes) {
    if (c->pinned) (void)hipHostFree(c->pinned);
    c->pinned = nullptr;
    c->pinned_bytes = 0;
    const size_t want = std::max<size_t>(bytes, 64 * 1024);
    CHECK_HIP(hipHostMalloc(&c->pinned, want, hipHostMallocDefault));
    c->pinned_bytes = want;
  }
  CHECK_HIP(hipMemcpyAsync(c->pinned, dev, bytes, hipMemcpyDeviceToHost, c->stream));
  CHECK_HIP(hipStreamSynchronize(c->stream));
  c->up_off = 0;   // the stream is drained: every staged upload has completed
  memcpy(host, c->pinned, bytes);
  return ok();
}

// Asynchronous host-to-device copy of `bytes` through the context's pinned upload stage: the
// source is copied into the stage at once, so it may go out of scope right away, and the
// stream need not be drained.  The stage is reused once the stream has been drained (a
// read-back); when it is full, the stream is drained here.
Err stage_upload(flsq_ctx* c, void* dev, const void* host, size_t bytes) {
  if (bytes == 0) return ok();
  const size_t need = (bytes + 255) / 256 * 256;
  if (c->up_off + need > c->up_bytes) {
    CHECK_HIP(hipStreamSynchronize(c->stream));
    c->up_off = 0;
    if (need > c->up_bytes) {
      if (c->up) (void)hipHostFree(c->up);
      c->up = nullptr;
      c->up_bytes = 0;
      const size_t want = std::max<size_t>(need, 4u << 20);
      CHECK_HIP(hipHostMalloc(&c->up, want, hipHostMallocDefault));
      c->up_bytes = want;
    }
  }
  char* dst = (char*)c->up + c->up_off;
  memcpy(dst, host, bytes);
  c->up_off += need;
  CHECK_HIP(hipMemcpyAsync(dev, dst, bytes, hipMemcpyHostToDevice, c->stream));
  return ok();
}

// ------------------------------------------------------------------ validation
Err check_basis(const flsq_basis* b) {
  if (!b) return fail(FLSQ_EINVAL, "basis is NULL");
  if (b->d < 1 || b->d > FLSQ_MAX_DIM) return fail(FLSQ_EINVAL, "basis.d = %d outside [1, %d]", b->d, FLSQ_MAX_DIM);
  if (b->n_feat < 1) return fail(FLSQ_EINVAL, "basis.n_feat = %d < 1", b->n_feat);
  if (!b->W || !b->b) return fail(FLSQ_EINVAL, "basis.W or basis.b is NULL");
  return ok();
}

Err check_op(const flsq_op& op, int d, int bi) {
  if (op.n_terms < 1 || op.n_terms > 32) return fail(FLSQ_EINVAL, "block %d: n_terms = %d outside [1, 32]", bi, op.n_terms);
  if (!op.terms) return fail(FLSQ_EINVAL, "block %d: terms is NULL", bi);
  for (int t = 0; t < op.n_terms; ++t) {
    for (int k = d; k < FLSQ_MAX_DIM; ++k)
      if (op.terms[t].alpha[k] != 0)
        return fail(FLSQ_EINVAL, "block %d term %d: multi-index has alpha[%d] = %d beyond d = %d", bi, t, k,
                    op.terms[t].alpha[k], d);
    if (!std::isfinite(op.terms[t].coef)) return fail(FLSQ_ENONFINITE, "block %d term %d: coefficient not finite", bi, t);
  }
  return ok();
}

Err check_blocks(const flsq_rows* blocks, int n_blocks, int d, bool need_rhs) {
  if (n_blocks < 1 || !blocks) return fail(FLSQ_EINVAL, "need at least one row block");
  if (n_blocks > 64) return fail(FLSQ_EINVAL, "at most 64 row blocks");
  int64_t P = 0;
  for (int i = 0; i < n_blocks; ++i) {
    const flsq_rows& r = blocks[i];
    if (r.n_rows < 0) return fail(FLSQ_EINVAL, "block %d: n_rows < 0", i);
    if (r.n_rows > 0 && !r.x) return fail(FLSQ_EINVAL, "block %d: x is NULL", i);
    if (need_rhs && r.n_rows > 0 && !r.rhs) return fail(FLSQ_EINVAL, "block %d: rhs is NULL", i);
    if (!std::isfinite(r.weight)) return fail(FLSQ_ENONFINITE, "block %d: weight not finite", i);
    CHECK_ERR(check_op(r.op, d, i));
    P += r.n_rows;
  }
  if (P < 1) return fail(FLSQ_EINVAL, "no rows");
  if (P > (int64_t)0x7fffffff) return fail(FLSQ_EINVAL, "more than 2^31 - 1 rows");
  return ok();
}

struct FiniteItem {
  const double* p;
  int64_t n;
  const char* what;
};

// NaN / Inf scan of several device arrays with one read-back of their counts.
Err check_finite_many(flsq_ctx* c, std::initializer_list<FiniteItem> items) {
  int* flags;
  const int m = (int)items.size();
  if (m > kFiniteBatchMax) return fail(FLSQ_EINVAL, "internal: too many finiteness checks");
  FiniteBatch fb{};
  fb.count = m;
  int k = 0;
  for (const FiniteItem& it : items) {
    fb.p[k] = it.n > 0 ? it.p : nullptr;
    fb.n[k] = it.n;
    ++k;
  }
  const int wgs = finite_batch_wgs(fb);
  CHECK_ERR(ws_get(c, "nf_flag", (size_t)kFiniteBatchMax * kFiniteBatchWgs, &flags));
  CHECK_HIP(launch_finite_batch(fb, flags, c->stream));
  int h[kFiniteBatchMax * kFiniteBatchWgs];
  CHECK_ERR(read_back(c, h, flags, sizeof(int) * m * wgs));
  k = 0;
  for (const FiniteItem& it : items) {
    for (int w = 0; w < wgs; ++w)
      if (h[k * wgs + w]) return fail(FLSQ_ENONFINITE, "%s contains NaN or Inf", it.what);
    ++k;
  }
  return ok();
}

Err check_finite_dev(flsq_ctx* c, const double* p, int64_t n, const char* what) {
  return check_finite_many(c, {FiniteItem{p, n, what}});
}

// ------------------------------------------------------------------ system setup
std::vector<Chunk> make_runs(const System& s, int run_rows) {
  std::vector<Chunk> v;
  for (int b = 0; b < s.n_blocks; ++b) {
    for (int64_t r = 0; r < s.rows[b]; r += run_rows) {
      Chunk c;
      c.row0 = (int32_t)(s.row0[b] + r);
      c.nrows = (int32_t)std::min<int64_t>(run_rows, s.rows[b] - r);
      c.block = b;
      c.pad = 0;
      v.push_back(c);
    }
  }
  return v;
}

Err build_system(flsq_ctx* c, System& s, const flsq_basis* basis, const flsq_rows* blocks, int n_blocks,
                 bool need_rhs) {
  CHECK_ERR(check_basis(basis));
  CHECK_ERR(check_blocks(blocks, n_blocks, basis->d, need_rhs));
  hipStream_t st = c->stream;
  s.d = basis->d;
  s.n = basis->n_feat;
  s.n_blocks = n_blocks;
  s.normalize = basis->normalize ? 1 : 0;
  s.norm = basis->normalize ? 1.0 / std::sqrt((double)s.n) : 1.0;
  s.row0.assign(n_blocks, 0);
  s.rows.assign(n_blocks, 0);
  s.weight.assign(n_blocks, 0.0);
  s.even.assign(n_blocks, 1);
  int64_t P = 0;
  for (int i = 0; i < n_blocks; ++i) {
    s.row0[i] = P;
    s.rows[i] = blocks[i].n_rows;
    s.weight[i] = blocks[i].weight;
    for (int t = 0; t < blocks[i].op.n_terms; ++t) {
      int ord = 0;
      for (int k = 0; k < s.d; ++k) ord += blocks[i].op.terms[t].alpha[k];
      if (ord & 1) s.even[i] = 0;
    }
    P += blocks[i].n_rows;
  }
  s.P = P;
  const int n = s.n, d = s.d;
  CHECK_HIP(s.Wt.ensure(sizeof(double) * d * n));
  CHECK_HIP(s.Wt32.ensure(sizeof(float) * d * n));
  CHECK_HIP(s.bvec.ensure(sizeof(double) * n));
  CHECK_HIP(s.Wrm.ensure(sizeof(double) * d * n));
  CHECK_HIP(s.Xrm.ensure(sizeof(double) * d * P));
  CHECK_HIP(s.amp.ensure(sizeof(double) * n_blocks * n));
  CHECK_HIP(s.ph.ensure(sizeof(double) * n_blocks * n));
  CHECK_HIP(s.amp32.ensure(sizeof(float) * n_blocks * n));
  CHECK_HIP(s.ph32.ensure(sizeof(float) * n_blocks * n));
  CHECK_HIP(s.Xt.ensure(sizeof(double) * d * P));
  CHECK_HIP(s.Xt32.ensure(sizeof(float) * d * P));
  CHECK_HIP(s.row_block.ensure(sizeof(int32_t) * P));
  CHECK_HIP(s.rhs_w.ensure(sizeof(double) * P));

  CHECK_HIP(launch_transpose(basis->W, n, d, s.Wt.as<double>(), s.Wt32.as<float>(), n, st));
  CHECK_HIP(hipMemcpyAsync(s.bvec.p, basis->b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  CHECK_HIP(hipMemcpyAsync(s.Wrm.p, basis->W, sizeof(double) * d * n, hipMemcpyDeviceToDevice, st));
  for (int i = 0; i < n_blocks; ++i) {
    const flsq_rows& r = blocks[i];
    OpTerms op;
    memset(&op, 0, sizeof op);
    op.n_terms = r.op.n_terms;
    for (int t = 0; t < op.n_terms; ++t) {
      op.coef[t] = r.op.terms[t].coef;
      for (int k = 0; k < kMaxDim; ++k) op.alpha[t][k] = r.op.terms[t].alpha[k];
    }
    CHECK_HIP(launch_prep_block(op, r.weight, s.norm, d, n, basis->W, basis->b, s.amp.as<double>() + (int64_t)i * n,
                                s.ph.as<double>() + (int64_t)i * n, s.amp32.as<float>() + (int64_t)i * n,
                                s.ph32.as<float>() + (int64_t)i * n, st));
  }
  for (int b0 = 0; b0 < n_blocks; b0 += kRowStageMax) {   // the rows of all blocks, a group per launch
    RowStage rs{};
    rs.block0 = b0;
    rs.count = std::min(kRowStageMax, n_blocks - b0);
    for (int b = 0; b < rs.count; ++b) {
      const flsq_rows& r = blocks[b0 + b];
      rs.x[b] = r.x;
      rs.rhs[b] = r.rhs;
      rs.weight[b] = r.weight;
      rs.row0[b] = s.row0[b0 + b];
      rs.rows[b] = r.n_rows;
    }
    CHECK_HIP(launch_stage_rows(rs, d, P, s.Xt.as<double>(), s.Xt32.as<float>(), s.Xrm.as<double>(),
                                s.row_block.as<int32_t>(), s.rhs_w.as<double>(), st));
  }
  CHECK_HIP(s.frec.ensure(sizeof(double) * n_blocks * n * frec_stride(d)));
  CHECK_HIP(launch_pack_features(s.Wrm.as<double>(), s.amp.as<double>(), s.ph.as<double>(), n_blocks, n, d,
                                 s.frec.as<double>(), st));
  // Gram chunks and pass runs (block-aligned), Gram stream-K plan
  std::vector<Chunk> ch = make_runs(s, gram_chunk_rows());
  std::vector<Chunk> rn = make_runs(s, pass_rows());
  std::vector<Chunk> wd = make_runs(s, wide_rows());
  s.n_chunks = (int)ch.size();
  s.n_runs = (int)rn.size();
  s.n_wide = (int)wd.size();
  CHECK_HIP(s.chunks.ensure(sizeof(Chunk) * ch.size()));
  CHECK_HIP(s.runs.ensure(sizeof(Chunk) * rn.size()));
  CHECK_HIP(s.wide.ensure(sizeof(Chunk) * wd.size()));
  CHECK_ERR(stage_upload(c, s.chunks.p, ch.data(), sizeof(Chunk) * ch.size()));
  CHECK_ERR(stage_upload(c, s.runs.p, rn.data(), sizeof(Chunk) * rn.size()));
  CHECK_ERR(stage_upload(c, s.wide.p, wd.data(), sizeof(Chunk) * wd.size()));

  const int T = gram_tile();
  s.nt = (n + T - 1) / T;
  const int64_t n_tiles = (int64_t)s.nt * (s.nt + 1) / 2;
  s.total_units = n_tiles * s.n_chunks;
  const int slots_hw = c->n_cu * std::max(1, gram_occupancy(0));
  const int64_t min_units = 8;
  int64_t nwg = std::min<int64_t>(slots_hw, (s.total_units + min_units - 1) / min_units);
  nwg = std::max<int64_t>(1, nwg);
  s.units_per_wg = (s.total_units + nwg - 1) / nwg;
  s.n_wg = (int)((s.total_units + s.units_per_wg - 1) / s.units_per_wg);
  s.max_seg = (int)((s.units_per_wg + s.n_chunks - 1) / s.n_chunks) + 1;
  std::vector<std::vector<int32_t>> per_tile(n_tiles);
  for (int w = 0; w < s.n_wg; ++w) {
    int64_t u = (int64_t)w * s.units_per_wg;
    const int64_t ue = std::min(u + s.units_per_wg, s.total_units);
    int seg = 0;
    while (u < ue) {
      const int64_t t = u / s.n_chunks;
      const int64_t c0 = u % s.n_chunks;
      const int64_t c1 = std::min<int64_t>(s.n_chunks, c0 + (ue - u));
      per_tile[t].push_back(w * s.max_seg + seg);
      ++seg;
      u += c1 - c0;
    }
    if (seg > s.max_seg) return fail(FLSQ_EINVAL, "internal: Gram plan segment overflow");
  }
  std::vector<int32_t> ptr(n_tiles + 1, 0), sl;
  for (int64_t t = 0; t < n_tiles; ++t) {
    ptr[t + 1] = ptr[t] + (int32_t)per_tile[t].size();
    sl.insert(sl.end(), per_tile[t].begin(), per_tile[t].end());
  }
  CHECK_HIP(s.slot_ptr.ensure(sizeof(int32_t) * ptr.size()));
  CHECK_HIP(s.slots.ensure(sizeof(int32_t) * std::max<size_t>(1, sl.size())));
  CHECK_ERR(stage_upload(c, s.slot_ptr.p, ptr.data(), sizeof(int32_t) * ptr.size()));
  CHECK_ERR(stage_upload(c, s.slots.p, sl.data(), sizeof(int32_t) * sl.size()));
  CHECK_ERR(check_finite_many(c, {FiniteItem{s.Xt.as<double>(), (int64_t)d * P, "collocation points"},
                                  FiniteItem{s.Wt.as<double>(), (int64_t)d * n, "W"},
                                  FiniteItem{s.bvec.as<double>(), n, "b"},
                                  FiniteItem{need_rhs ? s.rhs_w.as<double>() : nullptr, P, "right-hand side"}}));
  return ok();
}

// ------------------------------------------------------------------ Gram
// G (n x n) gets the Gram product of the stacked rows; upper triangle only unless mirror.
// Moduli of the int8 Gram: the 13 largest pairwise coprime odd numbers <= 255 (product
// ~2^102.2), with their inverses modulo each other for the Garner reconstruction.
const I8Moduli& i8_moduli() {
  static I8Moduli M = [] {
    I8Moduli m{};
    const int list[13] = {255, 253, 251, 247, 241, 239, 233, 229, 227, 223, 217, 211, 199};
    m.n_mod = 13;
    for (int t = 0; t < m.n_mod; ++t) {
      m.ip[t] = list[t];
      m.p[t] = list[t];
      m.inv_p[t] = 1.0 / list[t];
      m.pf[t] = (float)list[t];
      m.inv_pf[t] = 1.0f / (float)list[t];
    }
    for (int a = 0; a < m.n_mod; ++a)
      for (int k = 0; k < m.n_mod; ++k) {
        int inv = 0;
        if (a < k)
          for (int x = 1; x < m.ip[k]; ++x)
            if ((m.ip[a] % m.ip[k]) * x % m.ip[k] == 1) {
              inv = x;
              break;
            }
        m.cinv[a][k] = inv;
        m.cinvf[a][k] = (float)inv;
      }
    return m;
  }();
  return M;
}

// Integer bits B of the scaled entries: 2^(2B) P_pad < M / 2 keeps every Gram entry inside
// the range the residues determine; one bit of margin.
int i8_bits(int64_t P_pad) {
  const I8Moduli& M = i8_moduli();
  double log2m = 0.0;
  for (int t = 0; t < M.n_mod; ++t) log2m += std::log2((double)M.ip[t]);
  const int B = (int)std::floor((log2m - 1.0 - std::log2((double)P_pad)) / 2.0) - 1;
  return std::min(B, 52);
}

constexpr int64_t kI8MaxRows = 133000;   // 127^2 * rows < 2^31: exact int32 sums

// Y, cvec (nullable, both or neither): also form cvec = A^T Y from the entries the residue pass
// evaluates anyway.
Err run_gram_i8(flsq_ctx* c, const System& s, const double* rho, double* G, int mirror, double diag_add,
                const double* Y = nullptr, double* cvec = nullptr) {
  const int T = i8_tile(), KBR = i8_kblock();
  const int n = s.n;
  const int nt = (n + T - 1) / T, n_pad = nt * T, n_tiles = nt * (nt + 1) / 2;
  const int64_t P_pad = (s.P + 2 * KBR - 1) / (2 * KBR) * (2 * KBR);
  if (P_pad > kI8MaxRows)
    return fail(FLSQ_EINVAL, "INT8_CRT Gram supports at most %lld rows (got %lld)", (long long)kI8MaxRows,
                (long long)s.P);
  if ((int64_t)s.n_blocks * s.n >= INT32_MAX)
    return fail(FLSQ_EINVAL, "INT8_CRT Gram supports blocks x features below 2^31 (got %lld)",
                (long long)s.n_blocks * s.n);
  const int KB = (int)(P_pad / KBR);
  const I8Moduli& M = i8_moduli();
  const int B = i8_bits(P_pad);
  int8_t* R;
  int32_t* Gt;
  double *inv_scale, *scale, *rho_max;
  CHECK_ERR(ws_get(c, "i8_R", (size_t)M.n_mod * KB * n_pad * KBR, &R));
  CHECK_ERR(ws_get(c, "i8_Gt", (size_t)M.n_mod * n_tiles * T * T, &Gt));
  CHECK_ERR(ws_get(c, "i8_inv", (size_t)n, &inv_scale));
  CHECK_ERR(ws_get(c, "i8_scale", (size_t)n, &scale));
  CHECK_ERR(ws_get(c, "i8_rhomax", 1, &rho_max));
  const hipStream_t st = c->stream;
  int2* order;
  CHECK_ERR(ws_get(c, "i8_order", (size_t)n_tiles, &order));
  {
    std::vector<int2> h(n_tiles);
    i8_tile_order(nt, h.data());
    CHECK_ERR(stage_upload(c, order, h.data(), sizeof(int2) * n_tiles));
  }
  CHECK_HIP(launch_i8_scale(s.amp.as<double>(), s.n_blocks, n, rho, s.P, rho_max, B, inv_scale, scale, st));
  double* cpart = nullptr;
  if (cvec) CHECK_ERR(ws_get(c, "i8_cpart", (size_t)KB * n_pad, &cpart));
  CHECK_HIP(launch_i8_residues(s.geo(), rho, inv_scale, M, n_pad, KB, R, cvec ? Y : nullptr, cpart, cvec, st));
  I8GemmJob J;
  J.R = R;
  J.n_pad = n_pad;
  J.KB = KB;
  J.nt = nt;
  J.n_tiles = n_tiles;
  J.n_mod = M.n_mod;
  J.order = order;
  J.out = Gt;
  CHECK_HIP(hipEventRecord(c->ev0, st));
  CHECK_HIP(launch_gram_i8(J, st));
  CHECK_HIP(hipEventRecord(c->ev1, st));
  I8CrtJob Cj;
  Cj.M = M;
  Cj.Gt = Gt;
  Cj.scale = scale;
  Cj.n = n;
  Cj.nt = nt;
  Cj.n_tiles = n_tiles;
  Cj.G = G;
  Cj.mirror = mirror;
  Cj.diag_add = diag_add;
  CHECK_HIP(launch_i8_crt(Cj, st));
  return ok();
}

Err run_gram(flsq_ctx* c, const System& s, int prec, const double* rho, double* G, int mirror, double diag_add) {
  if (prec == FLSQ_PREC_INT8_CRT) return run_gram_i8(c, s, rho, G, mirror, diag_add);
  const int T = gram_tile();
  const size_t part_elems = (size_t)s.n_wg * s.max_seg * T * T;
  void* partial;
  if (prec == FLSQ_PREC_FP64) {
    double* p;
    CHECK_ERR(ws_get(c, "gram_partial", part_elems, &p));
    partial = p;
  } else {
    float* p;
    CHECK_ERR(ws_get(c, "gram_partial", part_elems, &p));
    partial = p;
  }
  float* rho32 = nullptr;
  if (rho && prec != FLSQ_PREC_FP64) {
    CHECK_ERR(ws_get(c, "rho32", (size_t)s.P, &rho32));
    CHECK_HIP(launch_to_f32(rho, rho32, s.P, c->stream));
  }
  GramLaunch L;
  L.g = s.geo();
  L.prec = prec == FLSQ_PREC_FP64 ? 0 : (prec == FLSQ_PREC_FP32_REFINE ? 1 : 2);
  L.rho = rho;
  L.rho32 = rho32;
  L.chunks = s.chunks.as<Chunk>();
  L.n_chunks = s.n_chunks;
  L.nt = s.nt;
  L.total_units = s.total_units;
  L.units_per_wg = s.units_per_wg;
  L.max_seg = s.max_seg;
  L.n_wg = s.n_wg;
  L.partial = partial;
  CHECK_HIP(hipEventRecord(c->ev0, c->stream));
  CHECK_HIP(launch_gram(L, c->stream));
  CHECK_HIP(hipEventRecord(c->ev1, c->stream));
  CHECK_HIP(launch_gram_reduce(L.prec, partial, s.slot_ptr.as<int32_t>(), s.slots.as<int32_t>(), s.nt, s.n, G, mirror,
                               diag_add, c->stream));
  return ok();
}

// ------------------------------------------------------------------ Cholesky and inverse factor
// Upload GEMM descriptors (host vector stays alive until the copy has completed).
Err upload_descs(flsq_ctx* c, const std::vector<GemmDesc>& h, GemmDesc** d_out) {
  GemmDesc* d;
  CHECK_ERR(ws_get(c, "gemm_descs", std::max<size_t>(1, h.size()), &d));
  CHECK_ERR(stage_upload(c, d, h.data(), sizeof(GemmDesc) * h.size()));
  *d_out = d;
  return ok();
}

// In-place upper Cholesky of G (only the upper triangle is read), and X = D U^{-1} (upper,
// zero below the diagonal; d nullable = ones), whose transpose W = U^{-T} is formed block row
// by block row inside the factorisation steps.  Pivots below boost (> 0) are raised to it
// (their count goes to *boosted_host); info_host > 0 at the first failed pivot (1-based:
// non-finite, or non-positive when boost = 0), the steps after a failure return at once, and
// X is then not written.
//
// status: device words, [0] the pivot status and [1] the raised pivots (ints), then `extra`
// more bytes that the same read-back brings to host_extra (the caller's values computed
// before the factorisation, so that it need not wait for them separately).
Err cholesky_inv(flsq_ctx* c, double* G, double* X, int n, const double* d, int* status, size_t extra,
                 void* host_extra, int* info_host, double boost, int* boosted_host) {
  int* info = status;
  double* W;
  hipStream_t st = c->stream;
  CHECK_ERR(ws_get(c, "chol_w", (size_t)n * n, &W));
  CHECK_HIP(hipMemsetAsync(info, 0, 2 * sizeof(int), st));
  CHECK_HIP(hipMemsetAsync(W, 0, sizeof(double) * n * n, st));
  // Block 0 and its block row first.  While the trailing matrix is large (the update launch then
  // spans several rounds of tiles and its HBM traffic dominates), block rows go in pairs k, k + 1:
  // the update of block row k + 1 alone by row k (with the factorisation of its diagonal block),
  // its solve, then the update of everything below by both rows at once (rank 128: the trailing
  // matrix is read and written once per pair), which also factors the next diagonal block; its
  // solve.  Smaller trailing matrices take one block row per step (measured: at N = 4096 the
  // pairs gain nothing there, at N = 8192 they save a quarter of the factorisation).
  constexpr int kPairTrailing = 4608;
  CHECK_HIP(launch_potrf(G, n, 0, info, boost, info + 1, st));
  CHECK_HIP(launch_trsm_row(G, W, n, 0, info, st));
  for (int k0 = 0; k0 + kNb < n;) {
    if (n - k0 - 2 * kNb >= kPairTrailing) {
      CHECK_HIP(launch_syrk_potrf(G, W, n, k0, kNb, k0 + 2 * kNb, info, boost, info + 1, st));
      CHECK_HIP(launch_trsm_row(G, W, n, k0 + kNb, info, st));
      CHECK_HIP(launch_syrk_potrf(G, W, n, k0, 2 * kNb, n, info, boost, info + 1, st));
      CHECK_HIP(launch_trsm_row(G, W, n, k0 + 2 * kNb, info, st));
      k0 += 2 * kNb;
    } else {
      CHECK_HIP(launch_syrk_potrf(G, W, n, k0, kNb, n, info, boost, info + 1, st));
      CHECK_HIP(launch_trsm_row(G, W, n, k0 + kNb, info, st));
      k0 += kNb;
    }
  }
  // X = D W^T is queued ahead of the status read; the kernel leaves X alone after a failed pivot
  CHECK_HIP(launch_inv_transpose(W, d, n, info, X, st));
  unsigned char hbuf[2 * sizeof(int) + 64];
  if (extra > 64) return fail(FLSQ_EINVAL, "internal: status read-back too long");
  CHECK_ERR(read_back(c, hbuf, info, 2 * sizeof(int) + extra));
  int hinfo[2];
  memcpy(hinfo, hbuf, sizeof hinfo);
  if (extra) memcpy(host_extra, hbuf + sizeof hinfo, extra);
  *info_host = hinfo[0];
  *boosted_host = hinfo[1];
  return ok();
}

// Z = (U^T U)^{-1} Y = X (X^T Y) for K columns (Y preserved, Z distinct from Y).
Err chol_solve(flsq_ctx* c, const double* X, int n, const double* Y, double* Z, int K) {
  hipStream_t st = c->stream;
  if (K == 1) {
    double *tmp, *work;
    CHECK_ERR(ws_get(c, "pa_tmp", (size_t)n, &tmp));
    CHECK_ERR(ws_get(c, "pa_work", precond_work_elems(n), &work));
    CHECK_HIP(launch_precond_apply(X, n, Y, tmp, work, Z, st));
    return ok();
  }
  // K > 1: T = X^T Y, then Z = X T, on the matrix cores with the contraction of each 16-row
  // tile split across workgroups (chunk partials summed in a fixed order).
  if (K > 64) return fail(FLSQ_EINVAL, "chol_solve: K = %d above 64", K);
  double *tmp, *part;
  CHECK_ERR(ws_get(c, "pa_tmpK", (size_t)n * K, &tmp));
  CHECK_ERR(ws_get(c, "pa_partK", chol_multi_work_elems(n, K), &part));
  CHECK_HIP(launch_chol_solve_multi(X, n, Y, K, tmp, part, Z, st));
  return ok();
}

// Factor the equilibrated system D (G_src + mu I) D + shift I (D = diag(G_src)^{-1/2}, so the
// scaled Gram has a unit diagonal), form X = U^{-1}, and return D X, whose outer product
// (D X)(D X)^T approximates (G + mu I)^{-1}.  The first attempt uses shift0 (0 for the FP64
// Gram).  Pivots of the equilibrated Gram below boost (> 0) are raised to it in place (their
// count goes to *boosted); a failed pivot (non-finite, or non-positive when boost = 0) retries
// the whole factorisation with growing shifts.
//
// Shift memory: when a factorisation needed retries, the context keeps a 64-bit fingerprint of
// the Gram's upper triangle with the shift that succeeded.  A later factorisation with the same
// size and settings whose Gram has the same fingerprint starts at that shift (*recalled = 1):
// the kernels are deterministic, so the attempts below it would fail as they did, and the
// result is the one the retries would reach.  Nothing is fingerprinted unless the last
// factorisation of this size needed a retry.
Err factor_with_retries(flsq_ctx* c, const double* Gsrc, double* U, double* X, int n, double mu, double shift0,
                        double* shift_used, int* retries, double boost = 0.0, int* boosted = nullptr,
                        int* recalled = nullptr) {
  double *stat, *d;
  unsigned long long* fp_part;
  // [0] the pivot status (two ints), [1] the largest diagonal entry, [2] the fingerprint
  CHECK_ERR(ws_get(c, "chol_status", 3, &stat));
  CHECK_ERR(ws_get(c, "eq_d", (size_t)n, &d));
  CHECK_ERR(ws_get(c, "fp_part", (size_t)n, &fp_part));
  int* status = reinterpret_cast<int*>(stat);
  double* dmax = stat + 1;
  unsigned long long* d_fp = reinterpret_cast<unsigned long long*>(stat + 2);
  // the entry for this size and these settings, if any (else the one a new entry replaces)
  ShiftMemo* memo = nullptr;
  for (ShiftMemo& m : c->shift_memo)
    if (m.valid && m.n == n && m.mu == mu && m.shift0 == shift0 && m.boost == boost) memo = &m;
  const bool memo_applies = memo && memo->shift > shift0;
  CHECK_HIP(launch_diag_max(Gsrc, n, dmax, c->stream));
  unsigned long long fp = 0;
  bool have_fp = false;
  if (memo_applies) {   // the starting shift depends on the fingerprint: wait for it
    CHECK_HIP(launch_fingerprint_upper(Gsrc, n, fp_part, d_fp, c->stream));
    double hv[2] = {0.0, 0.0};
    CHECK_ERR(read_back(c, hv, dmax, sizeof hv));
    if (!std::isfinite(hv[0])) return fail(FLSQ_ENONFINITE, "Gram diagonal is not finite");
    memcpy(&fp, &hv[1], sizeof fp);
    have_fp = true;
  }
  const bool recall = memo_applies && fp == memo->fp;
  if (recalled) *recalled = recall ? 1 : 0;
  double rel = recall ? memo->shift : shift0;
  *retries = 0;
  for (int attempt = 0; attempt < 8; ++attempt) {
    CHECK_HIP(launch_equilibrate(Gsrc, U, n, d, mu, rel, c->stream));
    int info = 0, nb = 0;
    double dm = 0.0;   // the diagonal's largest entry comes back with the first attempt's status
    CHECK_ERR(cholesky_inv(c, U, X, n, d, status, attempt == 0 && !memo_applies ? sizeof(double) : 0, &dm, &info,
                           boost, &nb));
    if (attempt == 0 && !memo_applies && !std::isfinite(dm))
      return fail(FLSQ_ENONFINITE, "Gram diagonal is not finite");
    if (info == 0) {
      *shift_used = rel;
      if (boosted) *boosted = nb;
      if (*retries > 0) {
        if (!have_fp) {
          CHECK_HIP(launch_fingerprint_upper(Gsrc, n, fp_part, d_fp, c->stream));
          CHECK_ERR(read_back(c, &fp, d_fp, sizeof fp));
        }
        if (!memo) {
          memo = &c->shift_memo[c->shift_memo_next];
          c->shift_memo_next = (c->shift_memo_next + 1) % 4;
        }
        memo->valid = true;
        memo->n = n;
        memo->mu = mu;
        memo->shift0 = shift0;
        memo->boost = boost;
        memo->fp = fp;
        memo->shift = rel;
      }
      return ok();
    }
    ++*retries;
    rel = (rel == 0.0) ? 1e-14 : rel * 10.0;
  }
  return fail(FLSQ_ENOTSPD, "Cholesky failed: Gram + mu I not positive definite after %d shift retries", *retries);
}

// Row pass with the workspace the many-column (MFMA) variant needs.
Err row_pass(flsq_ctx* c, const PassGeo& pg, const double* rho, const double* V, int K, const double* Y, double alpha,
             double beta_y, double* out, double* u_out = nullptr) {
  double* work = nullptr;
  const size_t we = rowpass_work_elems(pg, K);
  if (we) CHECK_ERR(ws_get(c, "rp_work", we, &work));
  CHECK_HIP(launch_rowpass_runs(pg, rho, V, K, Y, alpha, beta_y, out, c->stream, u_out, work));
  return ok();
}

// ------------------------------------------------------------------ CGLS refinement
// Minimise ||Y - A X||^2 + mu ||X||^2 column-wise, starting from X, preconditioned by U
// (U^T U ~ A^T A + mu I).  Y is P x K (weighted data).  On return X is refined.
struct RefineOut {
  int iters = 0;
  double grad0 = 0.0, grad = 0.0, last_step = 0.0;
  bool converged = false;
};

Err host_cols(flsq_ctx* c, const double* dev, int K, std::vector<double>& h) {
  h.resize(K);
  CHECK_ERR(read_back(c, h.data(), dev, sizeof(double) * K));
  return ok();
}

// Per-column scalars for the kernel arguments (K <= 64).
ColScalars cols(const std::vector<double>& h) {
  ColScalars c{};
  for (size_t k = 0; k < h.size() && k < 64; ++k) c.v[k] = h[k];
  return c;
}

// Bit k set where h[k] != 0 (K <= 64).
uint64_t col_mask(const std::vector<double>& h) {
  uint64_t m = 0;
  for (size_t k = 0; k < h.size() && k < 64; ++k)
    if (h[k] != 0.0) m |= 1ull << k;
  return m;
}

// Size of the change still to come, from the last two steps of a column: once the steps fall
// by at least 10x per iteration, the next one is predicted as step^2 / previous (geometric
// decay; CG usually converges faster still); otherwise the last step itself.  Stopping on the
// prediction saves the iteration that would only confirm it.
double predicted_step(int it, double prev, double cur) {
  if (it >= 1 && prev > 0.0 && cur <= 0.1 * prev) return cur * (cur / prev);
  return cur;
}

// Stopping rule (Section 2.4 prefers a solution-level change over the coefficient change,
// which is unreliable when features are nearly dependent): the relative change of u_N at
// the collocation rows of blocks with even-order operators, |alpha| ||H p|| <= tol ||H X||,
// where H p comes out of the same row pass as A p.  When no such rows exist (or K > 16)
// the change of the fitted values |alpha| ||A p|| <= tol ||Y|| is used instead.
// The operator the refinement applies: out = beta_y Y + alpha A V (and, optionally, the
// solution values u = H V on even-order blocks) and out = beta_v V + alpha A^T Y.
struct LsqOp {
  int n = 0;
  int64_t P = 0;
  virtual bool track_u(int K) const = 0;
  virtual Err apply(flsq_ctx* c, const double* V, int K, const double* Y, double alpha, double beta_y, double* out,
                    double* u_out) const = 0;
  virtual Err applyT(flsq_ctx* c, const double* Y, int K, const double* V, double alpha, double beta_v,
                     double* out) const = 0;
  virtual ~LsqOp() = default;
};

// A recomputed in FP64 by the row and column passes (matrix-free).
struct PassOp final : LsqOp {
  PassGeo pg;
  const double* rho;
  int n_runs;
  PassOp(const System& s, const double* r) : pg(s.pass()), rho(r), n_runs(s.n_runs) {
    n = s.n;
    P = s.P;
  }
  bool track_u(int K) const override { return K <= 16 && pg.even_mask != 0; }
  Err apply(flsq_ctx* c, const double* V, int K, const double* Y, double alpha, double beta_y, double* out,
            double* u_out) const override {
    return row_pass(c, pg, rho, V, K, Y, alpha, beta_y, out, u_out);
  }
  Err applyT(flsq_ctx* c, const double* Y, int K, const double* V, double alpha, double beta_v,
             double* out) const override {
    double* colwork;
    CHECK_ERR(ws_get(c, "cg_colwork", pass_work_elems(n, n_runs, K) + 64, &colwork));
    CHECK_HIP(launch_colpass_runs(pg, rho, Y, K, V, alpha, beta_v, out, colwork, c->stream));
    return ok();
  }
};

// A stored in HBM, row-major (P x n) and transposed (n x P); one column.
struct DenseOp final : LsqOp {
  const double* A;
  const double* At;
  DenseOp(const double* a, const double* at, int n_, int64_t P_) : A(a), At(at) {
    n = n_;
    P = P_;
  }
  bool track_u(int) const override { return false; }
  Err apply(flsq_ctx* c, const double* V, int K, const double* Y, double alpha, double beta_y, double* out,
            double*) const override {
    if (K != 1) return fail(FLSQ_EINVAL, "internal: the stored-matrix operator takes one column");
    CHECK_HIP(launch_rowdot(A, P, n, n, V, Y, alpha, beta_y, out, c->stream));
    return ok();
  }
  Err applyT(flsq_ctx* c, const double* Y, int K, const double* V, double alpha, double beta_v,
             double* out) const override {
    if (K != 1) return fail(FLSQ_EINVAL, "internal: the stored-matrix operator takes one column");
    CHECK_HIP(launch_rowdot(At, n, P, P, Y, V, alpha, beta_v, out, c->stream));
    return ok();
  }
};

// A and A^T kept by a factor object in FP64 MFMA operand order (launch_to_t16), for products
// with 2 .. 64 columns.
struct KeptOp final : LsqOp {
  const double* A16;
  const double* At16;
  KeptOp(const double* a, const double* at, int n_, int64_t P_) : A16(a), At16(at) {
    n = n_;
    P = P_;
  }
  bool track_u(int) const override { return false; }
  Err apply(flsq_ctx* c, const double* V, int K, const double* Y, double alpha, double beta_y, double* out,
            double*) const override {
    return many(c, A16, P, n, V, K, Y, alpha, beta_y, out);
  }
  Err applyT(flsq_ctx* c, const double* Y, int K, const double* V, double alpha, double beta_v,
             double* out) const override {
    return many(c, At16, n, P, Y, K, V, alpha, beta_v, out);
  }
  static Err many(flsq_ctx* c, const double* M16, int64_t rows, int64_t len, const double* B, int K, const double* B0,
                  double alpha, double beta, double* out) {
    double* part = nullptr;
    if (const size_t we = gemm_t16_work_elems(rows, len, K)) CHECK_ERR(ws_get(c, "t16_part", we, &part));
    CHECK_HIP(launch_gemm_t16(M16, rows, len, B, K, B0, alpha, beta, out, part, c->stream));
    return ok();
  }
};

// The operator of a factor object: the kept matrix for more than kDenseMinCols columns, the
// matrix-free passes otherwise (they also track the solution values the one-column stopping
// rule uses).
constexpr int kDenseMinCols = 16;
struct FactorOp {
  PassOp pass;
  KeptOp kept;
  bool has_kept;
  explicit FactorOp(const flsq_factor* F)
      : pass(F->sys, nullptr),
        kept(F->dense ? F->Ad.as<double>() : nullptr, F->dense ? F->Atd.as<double>() : nullptr, F->sys.n, F->sys.P),
        has_kept(F->dense) {}
  const LsqOp& for_k(int K) const {
    if (has_kept && K > kDenseMinCols) return kept;
    return pass;
  }
};

Err cgls_refine_op(flsq_ctx* c, const LsqOp& op, const double* Xi, double mu, const double* Y, int K, double* X,
                   int max_iter, double tol, bool want_grad0, bool want_grad, RefineOut* ro) {
  const int n = op.n;
  const int64_t P = op.P;
  const bool track_u = op.track_u(K);
  double *sres, *q, *g, *z, *p, *dots, *dwork, *uu = nullptr, *hq = nullptr;
  if (track_u) {
    CHECK_ERR(ws_get(c, "cg_u", (size_t)P * K, &uu));
    CHECK_ERR(ws_get(c, "cg_hq", (size_t)P * K, &hq));
  }
  CHECK_ERR(ws_get(c, "cg_s", (size_t)P * K, &sres));
  CHECK_ERR(ws_get(c, "cg_q", (size_t)P * K, &q));
  CHECK_ERR(ws_get(c, "cg_g", (size_t)n * K, &g));
  CHECK_ERR(ws_get(c, "cg_z", (size_t)n * K, &z));
  CHECK_ERR(ws_get(c, "cg_p", (size_t)n * K, &p));
  CHECK_ERR(ws_get(c, "cg_dots", (size_t)14 * K, &dots));
  CHECK_ERR(ws_get(c, "cg_dwork", (size_t)512 * K + 64, &dwork));
  hipStream_t st = c->stream;
  std::vector<double> tmp, stepn(K);

  // s = Y - A X ; g = A^T s - mu X ; u = H X
  CHECK_ERR(op.apply(c, X, K, Y, -1.0, 1.0, sres, uu));
  CHECK_ERR(op.applyT(c, sres, K, X, 1.0, -mu, g));
  // Per-column scalars on the device: gam | alpha | (unused) | qq | pp | hq.hq | u.u | s.s | X.X |
  // gam_new, then the starting values Y.Y | s.s | X.X | g.g (gam and gam_new alternate).  The host reads alpha, the step
  // norms and the objective once per iteration (the first read also brings the starting
  // values); the step lengths and the direction update never wait for it.
  double* d_gam = dots;
  double *d_alpha = dots + K, *d_qq = dots + 3 * K, *d_pp = dots + 4 * K;
  double *d_hh = dots + 5 * K, *d_uu = dots + 6 * K, *d_ss = dots + 7 * K, *d_xx = dots + 8 * K;
  double* d_gnew = dots + 9 * K;   // gam and gam_new trade places after every direction update
  double* d_start = dots + 10 * K;
  ro->iters = 0;
  ro->converged = (max_iter == 0);
  if (max_iter == 0) {
    if (want_grad0) {
      CHECK_HIP(launch_dot_cols(g, g, n, K, d_start + 3 * K, dwork, st));
      CHECK_ERR(host_cols(c, d_start + 3 * K, K, tmp));
      double m = 0;
      for (double v : tmp) m = std::max(m, std::sqrt(v));
      ro->grad0 = m;
    }
    ro->grad = ro->grad0;
    return ok();
  }
  // Objective J = ||Y - A X||^2 + mu ||X||^2 per column.  CGLS decreases it monotonically in
  // exact arithmetic; once rounding takes over (these systems are near the limit of FP64)
  // further steps can increase it and then diverge.  A column whose J rises stops (its
  // step is set to zero) and the best iterate seen is returned.
  std::vector<double> ynorm, Jbest(K), active(K, 1.0), improved(K, 0.0), relstep(K, 0.0),
      minstep(K, HUGE_VAL);
  std::vector<int> stagnant(K, 0);
  double* Xbest;
  CHECK_ERR(ws_get(c, "cg_xbest", (size_t)n * K, &Xbest));
  CHECK_HIP(hipMemcpyAsync(Xbest, X, sizeof(double) * n * K, hipMemcpyDeviceToDevice, st));
  {
    // starting values Y.Y | s.s | X.X | g.g in one batch
    DotBatch db{};
    db.K = K;
    db.count = want_grad0 ? 4 : 3;
    const double* v[4] = {Y, sres, X, g};
    const int64_t len[4] = {P, P, n, n};
    for (int b = 0; b < db.count; ++b) {
      db.x[b] = db.y[b] = v[b];
      db.n[b] = len[b];
      db.out[b] = d_start + b * K;
    }
    CHECK_HIP(launch_dot_batch(db, dwork, st));
  }
  ynorm.resize(K);
  CHECK_ERR(chol_solve(c, Xi, n, g, z, K));
  CHECK_HIP(launch_cg_direction(g, z, p, n, K, nullptr, d_gam, dwork, st));   // gam = g.z, p = z
  bool stalled_all = false;
  uint64_t keep_mask = 0;
  std::vector<double> hs(13 * K);
  for (int it = 0; it < max_iter; ++it) {
    // q = A p ; delta = ||q||^2 + mu ||p||^2 ; hq = H p ; alpha = gam / delta
    CHECK_ERR(op.apply(c, p, K, nullptr, 1.0, 0.0, q, hq));
    AxpyBatch ab{};
    ab.K = K;
    ab.count = track_u ? 3 : 2;
    ab.x[0] = p;
    ab.y[0] = X;
    ab.n[0] = n;
    ab.sign[0] = 1.0;
    ab.x[1] = q;
    ab.y[1] = sres;
    ab.n[1] = P;
    ab.sign[1] = -1.0;
    ab.x[2] = hq;
    ab.y[2] = uu;
    ab.n[2] = P;
    ab.sign[2] = 1.0;
    CgStepSmall cs{};
    {
      const double* pre[4] = {q, p, hq, uu};
      const int64_t pre_n[4] = {P, n, P, P};
      double* pre_out[4] = {d_qq, d_pp, d_hh, d_uu};
      cs.n_pre = track_u ? 4 : 2;
      for (int b = 0; b < cs.n_pre; ++b) {
        cs.pre[b] = pre[b];
        cs.pre_n[b] = pre_n[b];
        cs.pre_out[b] = pre_out[b];
      }
      cs.n_post = 2;
      cs.post[0] = sres;
      cs.post_n[0] = P;
      cs.post_out[0] = d_ss;
      cs.post[1] = X;
      cs.post_n[1] = n;
      cs.post_out[1] = d_xx;
      cs.gam = d_gam;
      cs.d1 = d_qq;
      cs.d2 = d_pp;
      cs.mu = mu;
      cs.active = col_mask(active);
      cs.alpha_out = d_alpha;
      cs.step = ab;
      cs.keep = Xbest;
      cs.keep_mask = keep_mask;
      cs.K = K;
    }
    if (cg_step_small_fits(cs)) {
      // small systems: the dots, the step and the dots after it in one workgroup
      CHECK_HIP(launch_cg_step_small(cs, st));
      keep_mask = 0;
    } else {
      {
        DotBatch db{};
        db.K = K;
        for (int b = 0; b < cs.n_pre; ++b) {
          db.x[b] = db.y[b] = cs.pre[b];
          db.n[b] = cs.pre_n[b];
          db.out[b] = cs.pre_out[b];
        }
        db.count = cs.n_pre;
        CHECK_HIP(launch_dot_batch(db, dwork, st));
      }
      // alpha = gam / delta and the step; X's columns improved by the previous step go to Xbest first
      CHECK_HIP(launch_cg_step(d_gam, d_qq, d_pp, mu, col_mask(active), d_alpha, ab, Xbest, keep_mask, st));
      keep_mask = 0;
      // objective after the step
      DotBatch db{};
      db.K = K;
      db.count = 2;
      db.x[0] = db.y[0] = sres;
      db.n[0] = P;
      db.out[0] = d_ss;
      db.x[1] = db.y[1] = X;
      db.n[1] = n;
      db.out[1] = d_xx;
      CHECK_HIP(launch_dot_batch(db, dwork, st));
    }
    // alpha .. X.X (8 K values), on the first iteration also the starting values (13 K)
    CHECK_ERR(read_back(c, hs.data(), d_alpha, sizeof(double) * (it == 0 ? 13 : 8) * K));
    if (it == 0) {
      const double* h0 = hs.data() + 9 * K;   // Y.Y | s.s | X.X | g.g
      for (int k = 0; k < K; ++k) {
        ynorm[k] = std::max(std::sqrt(h0[k]), 1e-300);
        Jbest[k] = h0[K + k] + mu * h0[2 * K + k];
      }
      if (want_grad0) {
        double m = 0;
        for (int k = 0; k < K; ++k) m = std::max(m, std::sqrt(h0[3 * K + k]));
        ro->grad0 = m;
      }
    }
    const double* h_alpha = hs.data();
    const double *h_qq = hs.data() + 2 * K, *h_hh = hs.data() + 4 * K, *h_uu = hs.data() + 5 * K;
    const double *h_ss = hs.data() + 6 * K, *h_xx = hs.data() + 7 * K;
    double worst = 0.0, worst_pred = 0.0;
    for (int k = 0; k < K; ++k) {
      if (active[k] == 0.0) continue;
      const double prev = relstep[k];
      if (track_u && h_uu[k] > 0.0) {
        stepn[k] = std::fabs(h_alpha[k]) * std::sqrt(h_hh[k]);
        relstep[k] = stepn[k] / std::sqrt(h_uu[k]);
      } else {
        stepn[k] = std::fabs(h_alpha[k]) * std::sqrt(h_qq[k]);
        relstep[k] = stepn[k] / ynorm[k];
      }
      worst = std::max(worst, relstep[k]);
      worst_pred = std::max(worst_pred, predicted_step(it, prev, relstep[k]));
    }
    ro->iters = it + 1;
    ro->last_step = worst;
    // Keep the best iterate, stop columns whose objective rose.  A column also stops once,
    // for two iterations in a row, neither its objective dropped by more than a few units in
    // the last place nor its step shrank below half the smallest step so far: FP64 no longer
    // resolves its progress.  The objective alone is not enough: it is quadratic in the
    // error, so it stops resolving progress at a relative error of about the square root of
    // the unit roundoff, while the step keeps shrinking until the rounding floor.  An
    // objective within a few ulps of the best counts as a tie and takes the newer iterate.
    int n_active = 0;
    for (int k = 0; k < K; ++k) {
      improved[k] = 0.0;
      if (active[k] == 0.0) continue;
      const double J = h_ss[k] + mu * h_xx[k];
      const double ulps = 4.0 * DBL_EPSILON * Jbest[k];
      const bool resolved = (Jbest[k] - J) > ulps || relstep[k] < 0.5 * minstep[k];
      minstep[k] = std::min(minstep[k], relstep[k]);
      if (J <= Jbest[k] + ulps) {
        Jbest[k] = std::min(Jbest[k], J);
        improved[k] = 1.0;
      } else if (J > Jbest[k] * (1.0 + 1e-12)) {
        active[k] = 0.0;
      }
      stagnant[k] = resolved ? 0 : stagnant[k] + 1;
      if (stagnant[k] >= 2) active[k] = 0.0;
      if (active[k] > 0.0) ++n_active;
    }
    keep_mask = col_mask(improved);   // copied by the next step's launch, or below
    if (worst_pred <= tol) {
      ro->converged = true;
      break;
    }
    if (n_active == 0) {
      stalled_all = true;
      break;
    }
    if (it + 1 == max_iter) break;
    // g = A^T s - mu X ; z = M^{-1} g ; beta = (g.z) / gam ; p = z + beta p
    CHECK_ERR(op.applyT(c, sres, K, X, 1.0, -mu, g));
    CHECK_ERR(chol_solve(c, Xi, n, g, z, K));
    CHECK_HIP(launch_cg_direction(g, z, p, n, K, d_gam, d_gnew, dwork, st));
    std::swap(d_gam, d_gnew);
  }
  if (keep_mask) CHECK_HIP(launch_select_cols(X, Xbest, n, K, keep_mask, st));
  // return the best iterate of every column; the recurrence residual is recomputed
  CHECK_HIP(hipMemcpyAsync(X, Xbest, sizeof(double) * n * K, hipMemcpyDeviceToDevice, st));
  if (stalled_all) ro->converged = true;   // no further progress is possible in FP64
  if (want_grad) {
    CHECK_ERR(op.apply(c, X, K, Y, -1.0, 1.0, sres, nullptr));
    CHECK_ERR(op.applyT(c, sres, K, X, 1.0, -mu, g));
    CHECK_HIP(launch_dot_cols(g, g, n, K, dots, dwork, st));
    CHECK_ERR(host_cols(c, dots, K, tmp));
    double m = 0;
    for (double v : tmp) m = std::max(m, std::sqrt(v));
    ro->grad = m;
  }
  return ok();
}

Err cgls_refine(flsq_ctx* c, const System& s, const double* rho, const double* Xi, double mu, const double* Y, int K,
                double* X, int max_iter, double tol, bool want_grad0, bool want_grad, RefineOut* ro) {
  return cgls_refine_op(c, PassOp(s, rho), Xi, mu, Y, K, X, max_iter, tol, want_grad0, want_grad, ro);
}

// ------------------------------------------------------------------ one full solve on a built system
struct SolveParams {
  double mu = 0.0;
  int prec = FLSQ_PREC_FP64;
  int max_refine = 0;
  double refine_tol = 0.0;
  double shift_rel = 0.0;
  bool report_grad = false;
  int second_pass = 0;
  double pivot_boost = 0.0;   // > 0 raises low pivots in place, 0 retries with shifts
  bool store_matrix = false;  // factor objects: keep A and A^T in HBM for the many-column products
};

// Boost of the second pass's factorisation (its Gram is far better conditioned than the first).
constexpr double kSecondPassPivotBoost = 0.0;

SolveParams params_of(const flsq_solve_opts* o) {
  SolveParams p;
  if (o) {
    p.mu = o->mu;
    p.prec = o->prec;
    p.max_refine = o->max_refine;
    p.refine_tol = o->refine_tol;
    p.shift_rel = o->shift_rel;
    p.report_grad = o->report_grad != 0;
    p.second_pass = o->second_pass;
    p.pivot_boost = o->pivot_boost;
    p.store_matrix = o->store_matrix != 0;
  }
  return p;
}

Err check_params(const SolveParams& p) {
  if (!(p.mu >= 0.0) || !std::isfinite(p.mu)) return fail(FLSQ_EINVAL, "mu must be finite and >= 0");
  if (p.prec != FLSQ_PREC_FP64 && p.prec != FLSQ_PREC_FP32_REFINE && p.prec != FLSQ_PREC_BF16X3_REFINE &&
      p.prec != FLSQ_PREC_INT8_CRT)
    return fail(FLSQ_EINVAL, "unknown precision %d", p.prec);
  if (p.max_refine < 0 || p.max_refine > 100000) return fail(FLSQ_EINVAL, "max_refine out of range");
  if (!(p.refine_tol >= 0.0)) return fail(FLSQ_EINVAL, "refine_tol must be >= 0");
  if (!(p.shift_rel >= 0.0) || p.shift_rel > 1.0) return fail(FLSQ_EINVAL, "shift_rel must be in [0, 1]");
  if (p.second_pass < -1 || p.second_pass > 1) return fail(FLSQ_EINVAL, "second_pass must be -1, 0 or 1");
  if (!(p.pivot_boost >= 0.0 && p.pivot_boost < 1.0)) return fail(FLSQ_EINVAL, "pivot_boost must be in [0, 1)");
  return ok();
}

// Second factorisation pass (the Cholesky-QR idea applied to the regularised system).  The
// first factor's inverse Xi (n x n, upper, equilibration folded in) makes B Xi, B = [A; sqrt(mu) I],
// much better conditioned than B.  Its Gram Q^T Q + mu Xi^T Xi is formed from Q = A Xi itself
// (stored in HBM), not from the rounded Gram of A, factored again (X2), and Xi becomes Xi X2.
// Where the first Cholesky needed a diagonal shift, the refinement then converges in a few
// steps instead of tens.  A: P x n row-major in HBM.
Err second_pass_factor(flsq_ctx* c, const double* A, int64_t P, int n, double mu, double* Xi, double* shift2,
                       int* retries2, bool* applied) {
  *applied = true;
  hipStream_t st = c->stream;
  double *Q, *Qt, *G2, *U, *X2, *Xn, *work;
  CHECK_ERR(ws_get(c, "sp_Q", (size_t)P * n, &Q));
  CHECK_ERR(ws_get(c, "sp_G2", (size_t)n * n, &G2));
  CHECK_ERR(ws_get(c, "Ufac", (size_t)n * n, &U));
  CHECK_ERR(ws_get(c, "sp_X2", (size_t)n * n, &X2));
  CHECK_ERR(ws_get(c, "sp_Xn", (size_t)n * n, &Xn));
  const size_t we = (size_t)8 * n * n;
  CHECK_ERR(ws_get(c, "sp_work", we, &work));
  CHECK_ERR(ws_get(c, "sp_Qt", (size_t)P * n, &Qt));
  const int n_split = 1;
  std::vector<GemmDesc> h(n_split + 3);
  for (auto& g : h) memset(&g, 0, sizeof g);
  GemmDesc& dq = h[0];   // Q = A Xi, Xi upper triangular
  dq.A = A;
  dq.lda = n;
  dq.B = Xi;
  dq.ldb = n;
  dq.C = Q;
  dq.ldc = n;
  dq.M = (int)P;
  dq.N = n;
  dq.K = n;
  dq.tri = 1;
  {   // G2 = Q^T Q from the transposed copy (K = P split across workgroups)
    GemmDesc& g = h[1];
    g.A = Qt;
    g.lda = (int)P;
    g.B = Q;
    g.ldb = n;
    g.C = G2;
    g.ldc = n;
    g.M = n;
    g.N = n;
    g.K = (int)P;
  }
  GemmDesc& dx = h[1 + n_split];   // G2 += mu Xi^T Xi
  dx.A = Xi;
  dx.lda = n;
  dx.B = Xi;
  dx.ldb = n;
  dx.C = G2;
  dx.ldc = n;
  dx.M = n;
  dx.N = n;
  dx.K = n;
  GemmDesc& dm = h[2 + n_split];   // Xn = Xi X2, X2 upper triangular
  dm.A = Xi;
  dm.lda = n;
  dm.B = X2;
  dm.ldb = n;
  dm.C = Xn;
  dm.ldc = n;
  dm.M = n;
  dm.N = n;
  dm.K = n;
  dm.tri = 1;
  GemmDesc* d;
  CHECK_ERR(ws_get(c, "sp_descs", h.size(), &d));
  CHECK_ERR(stage_upload(c, d, h.data(), sizeof(GemmDesc) * h.size()));
  CHECK_HIP(launch_gemm_tri(d, 1, (int)P, n, n, 1.0, work, we, st));
  CHECK_HIP(launch_transpose_f64(Q, P, n, Qt, st));
  CHECK_HIP(launch_gemm_tri(d + 1, 1, n, n, (int)P, 1.0, work, we, st));
  CHECK_HIP(launch_gemm_batched(d + 1 + n_split, 1, n, n, mu, 1.0, 1, st));
  int boosted2 = 0;
  Err fe = factor_with_retries(c, G2, U, X2, n, 0.0, 0.0, shift2, retries2, kSecondPassPivotBoost, &boosted2);
  if (fe.st == FLSQ_ENOTSPD) {   // the first factor stays in use
    *applied = false;
    return ok();
  }
  CHECK_ERR(fe);
  CHECK_HIP(launch_gemm_tri(d + 2 + n_split, 1, n, n, n, 1.0, work, we, st));
  CHECK_HIP(hipMemcpyAsync(Xi, Xn, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
  return ok();
}

bool second_pass_allowed(const SolveParams& sp, const double*, int64_t P, int n) {
  if (sp.second_pass < 0) return false;
  if (sp.prec != FLSQ_PREC_FP64 && sp.prec != FLSQ_PREC_INT8_CRT) return false;
  return sp.second_pass > 0 || 2.0 * (double)P * n * n <= 2e11;
}

// Taken at factorisation: always when asked for, automatically when the first factor needed a shift.
bool want_second_pass(const SolveParams& sp, int retries, const double* rho, int64_t P, int n) {
  if (!second_pass_allowed(sp, rho, P, n)) return false;
  return sp.second_pass > 0 || retries > 0;
}

// Steps of refinement after which an automatic second pass not taken at factorisation is taken
// anyway (an unshifted factor can still leave tens of CG steps on a nearly singular Gram), when
// 2 P N^2 is at most kLazySecondPassFlops: the pass costs about 1.5 such products plus a
// Cholesky, and beyond this size tens of CG steps are cheaper.
constexpr int kLazySecondPassIters = 8;
constexpr double kLazySecondPassFlops = 4e10;

// Refinement that takes the automatic second pass late: at most kLazySecondPassIters steps with
// the first factor; if they do not converge, re-factor through the preconditioned matrix
// (make_A() gives A, P x n in HBM) and continue from the current iterate.
template <class MakeA>
Err refine_lazy(flsq_ctx* c, const LsqOp& op, const SolveParams& sp, bool lazy, MakeA make_A, double* Xi,
                const double* Yw, int K, double* X, bool want_grad0, bool want_grad, RefineOut* ro, bool* second,
                double* t_second) {
  const int first = lazy ? std::min(sp.max_refine, kLazySecondPassIters) : sp.max_refine;
  CHECK_ERR(cgls_refine_op(c, op, Xi, sp.mu, Yw, K, X, first, sp.refine_tol, want_grad0, want_grad && !lazy, ro));
  if (!lazy || ro->converged || sp.max_refine <= first) {
    if (lazy && want_grad) {   // the gradient at the returned point was not taken in the short run
      RefineOut r2;
      CHECK_ERR(cgls_refine_op(c, op, Xi, sp.mu, Yw, K, X, 0, sp.refine_tol, true, false, &r2));
      ro->grad = r2.grad0;
    }
    return ok();
  }
  const double t0 = now_ms();
  const double* A = nullptr;
  CHECK_ERR(make_A(&A));
  double shift2 = 0.0;
  int retries2 = 0;
  bool applied = false;
  CHECK_ERR(second_pass_factor(c, A, op.P, op.n, sp.mu, Xi, &shift2, &retries2, &applied));
  CHECK_HIP(hipStreamSynchronize(c->stream));
  *second = applied;
  *t_second = now_ms() - t0;
  RefineOut r2;
  CHECK_ERR(cgls_refine_op(c, op, Xi, sp.mu, Yw, K, X, sp.max_refine - ro->iters, sp.refine_tol, false, want_grad,
                           &r2));
  ro->iters += r2.iters;
  ro->converged = r2.converged;
  ro->last_step = r2.last_step;
  ro->grad = want_grad ? r2.grad : ro->grad0;
  return ok();
}

// Gram, Cholesky, and the inverse factor Xi = U^{-1} (the preconditioner is Xi Xi^T).
// Y1, c1 (nullable): a single right-hand side whose c1 = A^T Y1 the INT8_CRT Gram forms on the way
// (*c1_formed tells whether it did; other precisions leave it to the caller).
Err gram_and_factor(flsq_ctx* c, const System& s, const double* rho, const SolveParams& sp, double* Xi,
                    flsq_solve_info* info, bool* second_out = nullptr, const double* Y1 = nullptr,
                    double* c1 = nullptr, bool* c1_formed = nullptr) {
  const int n = s.n;
  double *G, *U;
  CHECK_ERR(ws_get(c, "G", (size_t)n * n, &G));
  CHECK_ERR(ws_get(c, "Ufac", (size_t)n * n, &U));
  const double t0 = now_ms();
  const bool fold_c = sp.prec == FLSQ_PREC_INT8_CRT && Y1 && c1;
  // No host wait between the Gram and the factorisation: their kernels queue back to back, and
  // the first wait is the factorisation's status read (the phase times come from events).
  CHECK_HIP(hipEventRecord(c->ev_g0, c->stream));
  if (fold_c)
    CHECK_ERR(run_gram_i8(c, s, rho, G, 0, 0.0, Y1, c1));
  else
    CHECK_ERR(run_gram(c, s, sp.prec, rho, G, 0, 0.0));
  CHECK_HIP(hipEventRecord(c->ev_g1, c->stream));
  if (c1_formed) *c1_formed = fold_c;
  double shift = 0.0;
  int retries = 0;
  const bool exact_gram = sp.prec == FLSQ_PREC_FP64 || sp.prec == FLSQ_PREC_INT8_CRT;
  const double rel0 = exact_gram ? sp.shift_rel : (sp.shift_rel > 0.0 ? sp.shift_rel : 1e-6);
  int boosted = 0, recalled = 0;
  CHECK_ERR(factor_with_retries(c, G, U, Xi, n, sp.mu, rel0, &shift, &retries, sp.pivot_boost, &boosted, &recalled));
  // the status read waited for the Gram's events
  float gms = 0.f, kms = 0.f;
  CHECK_HIP(hipEventElapsedTime(&gms, c->ev_g0, c->ev_g1));
  CHECK_HIP(hipEventElapsedTime(&kms, c->ev0, c->ev1));
  c->last_gram_kernel_ms = kms;
  const double t2a = now_ms();
  bool second = false;
  // a recalled shift counts as the retries it skipped (the same factor, so the same decision)
  if (want_second_pass(sp, retries + recalled + (boosted > 0 ? 1 : 0), rho, s.P, n)) {
    double* A;
    CHECK_ERR(ws_get(c, "sp_A", (size_t)s.P * n, &A));
    CHECK_HIP(launch_assemble(s.geo(), 0, A, c->stream));
    if (rho) CHECK_HIP(launch_add_rho(s.geo(), rho, A, c->stream));
    double shift2 = 0.0;
    int retries2 = 0;
    CHECK_ERR(second_pass_factor(c, A, s.P, n, sp.mu, Xi, &shift2, &retries2, &second));
    CHECK_HIP(hipStreamSynchronize(c->stream));
    retries += retries2;
  }
  if (second_out) *second_out = second;
  CHECK_HIP(hipStreamSynchronize(c->stream));   // the inverse factor's kernels belong to this phase
  const double t2 = now_ms();
  if (info) {
    info->t_gram_ms = gms;
    info->t_chol_ms = std::max(t2 - t0 - gms, 0.0);
    info->shift = shift;
    info->chol_retries = retries;
    info->boosted_pivots = boosted;
    info->shift_recalled = recalled;
    info->t_gram_kernel_ms = c->last_gram_kernel_ms;
    info->second_pass = second ? 1 : 0;
    info->t_second_pass_ms = second ? t2 - t2a : 0.0;
  }
  return ok();
}

// Solve with the factor already held in Xinv (formed by an earlier solve on a system with the
// same features, such as the previous Newton step's): it preconditions at most reuse_iters CG
// steps; if they do not converge, the system's own Gram and factor are formed, with the second
// pass so that the new factor serves later solves as well, and CG continues from the iterate
// reached.  The result meets the same stopping rule as a solve that factors first.
Err solve_reusing_factor(flsq_ctx* c, const System& s, const double* rho, const SolveParams& sp, const double* Yw,
                         int K, double* X, int reuse_iters, flsq_solve_info* info, bool* converged, bool* factored) {
  const int n = s.n;
  double* Xi;
  CHECK_ERR(ws_get(c, "Xinv", (size_t)n * n, &Xi));
  const double t0 = now_ms();
  double *cvec, *colwork;
  CHECK_ERR(ws_get(c, "cvec", (size_t)n * K, &cvec));
  CHECK_ERR(ws_get(c, "colwork0", pass_work_elems(n, s.n_runs, K) + 64, &colwork));
  CHECK_HIP(launch_colpass_runs(s.pass(), rho, Yw, K, nullptr, 1.0, 0.0, cvec, colwork, c->stream));
  CHECK_ERR(chol_solve(c, Xi, n, cvec, X, K));
  const PassOp op(s, rho);
  RefineOut ro;
  CHECK_ERR(cgls_refine_op(c, op, Xi, sp.mu, Yw, K, X, std::min(reuse_iters, sp.max_refine), sp.refine_tol,
                           info != nullptr, false, &ro));
  *factored = false;
  if (info) memset(info, 0, sizeof *info);
  double t_fac = 0.0;
  if (!ro.converged && ro.iters < sp.max_refine) {
    SolveParams sp2 = sp;
    sp2.second_pass = 1;
    const double tf = now_ms();
    CHECK_ERR(gram_and_factor(c, s, rho, sp2, Xi, info));
    t_fac = now_ms() - tf;
    *factored = true;
    RefineOut r2;
    CHECK_ERR(cgls_refine_op(c, op, Xi, sp.mu, Yw, K, X, sp.max_refine - ro.iters, sp.refine_tol, false, false, &r2));
    ro.iters += r2.iters;
    ro.converged = r2.converged;
    ro.last_step = r2.last_step;
  }
  CHECK_HIP(hipStreamSynchronize(c->stream));
  if (info) {
    info->refine_iters = ro.iters;
    info->grad_norm0 = ro.grad0;
    info->grad_norm = ro.grad0;
    info->last_step_rel = ro.last_step;
    info->t_total_ms = now_ms() - t0;
    info->t_refine_ms = info->t_total_ms - t_fac;
  }
  if (converged) *converged = ro.converged;
  return ok();
}

Err solve_on_system(flsq_ctx* c, const System& s, const double* rho, const SolveParams& sp, const double* Yw, int K,
                    double* X, flsq_solve_info* info, bool* converged) {
  const int n = s.n;
  double* Xi;
  CHECK_ERR(ws_get(c, "Xinv", (size_t)n * n, &Xi));
  // X0 = (U^T U)^{-1} A^T Y; with one right-hand side the INT8_CRT Gram's residue pass forms A^T Y
  double *cvec, *colwork;
  CHECK_ERR(ws_get(c, "cvec", (size_t)n * K, &cvec));
  bool eager = false, c_formed = false;
  CHECK_ERR(gram_and_factor(c, s, rho, sp, Xi, info, &eager, K == 1 ? Yw : nullptr, K == 1 ? cvec : nullptr,
                            &c_formed));
  const double t1 = now_ms();
  if (!c_formed) {
    CHECK_ERR(ws_get(c, "colwork0", pass_work_elems(n, s.n_runs, K) + 64, &colwork));
    CHECK_HIP(launch_colpass_runs(s.pass(), rho, Yw, K, nullptr, 1.0, 0.0, cvec, colwork, c->stream));
  }
  CHECK_ERR(chol_solve(c, Xi, n, cvec, X, K));
  RefineOut ro;
  const bool lazy = sp.second_pass == 0 && !eager && second_pass_allowed(sp, rho, s.P, n) &&
                    2.0 * (double)s.P * n * n <= kLazySecondPassFlops;
  bool second = false;
  double t_second = 0.0;
  auto make_A = [&](const double** A) -> Err {
    double* buf;
    CHECK_ERR(ws_get(c, "sp_A", (size_t)s.P * n, &buf));
    CHECK_HIP(launch_assemble(s.geo(), 0, buf, c->stream));
    if (rho) CHECK_HIP(launch_add_rho(s.geo(), rho, buf, c->stream));
    *A = buf;
    return ok();
  };
  CHECK_ERR(refine_lazy(c, PassOp(s, rho), sp, lazy, make_A, Xi, Yw, K, X, info != nullptr,
                        info != nullptr && sp.report_grad, &ro, &second, &t_second));
  // no wait here: the refinement's last read-back waited for its passes, and the best-iterate
  // copies queued after it complete before the caller's next read (every caller ends in one)
  const double t2 = now_ms();
  if (info) {
    info->refine_iters = ro.iters;
    info->grad_norm0 = ro.grad0;
    info->grad_norm = ro.grad;
    info->last_step_rel = ro.last_step;
    info->t_refine_ms = t2 - t1;
    if (second) {
      info->second_pass = 1;
      info->t_second_pass_ms = t_second;
    }
  }
  if (converged) *converged = ro.converged;
  return ok();
}

// Build the system of `blocks` into F and factor it (the body of flsq_factorize, reusable on an
// existing factor object so that repeated calls keep its device buffers).
Err factor_into(flsq_ctx* c, flsq_factor* f, const flsq_basis* basis, const flsq_rows* blocks, int n_blocks,
                const SolveParams& sp, flsq_solve_info* info) {
  f->device = c->device;
  CHECK_ERR(build_system(c, f->sys, basis, blocks, n_blocks, false));
  if (f->Xinv.ensure(sizeof(double) * f->sys.n * f->sys.n) != hipSuccess)
    return fail(FLSQ_ENOMEM, "factor allocation failed");
  flsq_solve_info local;
  memset(&local, 0, sizeof local);
  CHECK_ERR(gram_and_factor(c, f->sys, nullptr, sp, f->Xinv.as<double>(), info ? info : &local));
  f->dense = false;
  if (sp.store_matrix) {
    // A assembled row-major into the context's workspace, then kept as A and A^T in MFMA
    // operand order
    const System& s = f->sys;
    const size_t ba = sizeof(double) * t16_elems(s.P, s.n), bt = sizeof(double) * t16_elems(s.n, s.P);
    if (f->Ad.ensure(ba) != hipSuccess || f->Atd.ensure(bt) != hipSuccess)
      return fail(FLSQ_ENOMEM, "keeping the %lld x %d matrix needs %zu + %zu bytes", (long long)s.P, s.n, ba, bt);
    double* A;
    CHECK_ERR(ws_get(c, "sp_A", (size_t)s.P * s.n, &A));
    CHECK_HIP(launch_assemble(s.geo(), 0, A, c->stream));
    CHECK_HIP(launch_to_t16(A, s.P, s.n, 0, f->Ad.as<double>(), c->stream));
    CHECK_HIP(launch_to_t16(A, s.n, s.P, 1, f->Atd.as<double>(), c->stream));
    CHECK_HIP(hipStreamSynchronize(c->stream));
    f->dense = true;
  } else {
    f->Ad.release();
    f->Atd.release();
  }
  f->mu = sp.mu;
  f->shift = info ? info->shift : local.shift;
  f->max_refine = sp.max_refine;
  f->refine_tol = sp.refine_tol;
  f->report_grad = sp.report_grad;
  // derived geometries and the observation operator of earlier calls no longer match
  f->rep_key = nullptr;
  f->rep_nobs = f->rep_nsrc = -1;
  f->obs_key = nullptr;
  f->obs_n = -1;
  f->akap_rows = -1;
  f->akap_dims = -1;
  return ok();
}

flsq_status finish(flsq_ctx* c, const Err& e) {
  if (c) c->err = e.msg;
  return e.st;
}

// Evaluation staging (per-feature transposed W, folded coefficients, FP32 copies, the multi-index
// list), carved from one region in 256-byte pieces.
struct EvalScratch {
  double *Wt, *coef;
  float *Wt32, *coef32, *b32;
  uint8_t* al;
};

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t eval_scratch_bytes(int d, int n, int n_alpha) {
  return align256(sizeof(double) * d * n) + align256(sizeof(double) * n_alpha * n) + align256(sizeof(float) * d * n) +
         align256(sizeof(float) * n_alpha * n) + align256(sizeof(float) * n) + align256((size_t)n_alpha * d);
}

EvalScratch carve_eval(unsigned char* base, int d, int n, int n_alpha) {
  EvalScratch e;
  size_t off = 0;
  e.Wt = reinterpret_cast<double*>(base + off);
  off += align256(sizeof(double) * d * n);
  e.coef = reinterpret_cast<double*>(base + off);
  off += align256(sizeof(double) * n_alpha * n);
  e.Wt32 = reinterpret_cast<float*>(base + off);
  off += align256(sizeof(float) * d * n);
  e.coef32 = reinterpret_cast<float*>(base + off);
  off += align256(sizeof(float) * n_alpha * n);
  e.b32 = reinterpret_cast<float*>(base + off);
  off += align256(sizeof(float) * n);
  e.al = base + off;
  return e;
}

// flsq_evaluate and flsq_evaluate_noalloc: the same kernels; the staging comes from the context's
// workspace (allocated on first use or growth) or from this device's static scratch (no allocation;
// sizes beyond it are rejected).  Every staged value is written before it is read, so the scratch
// needs no clearing between calls.
flsq_status evaluate_entry(flsq_ctx* ctx, const flsq_basis* basis, const double* beta, int64_t n_q, const void* xq,
                           int32_t xq_is_fp32, const uint8_t* alphas, int32_t n_alpha, void* out, bool no_alloc) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  Err e = check_basis(basis);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (!beta || (n_q > 0 && (!xq || !out))) return finish(ctx, fail(FLSQ_EINVAL, "NULL beta, xq or out"));
  if (n_q < 0) return finish(ctx, fail(FLSQ_EINVAL, "n_q < 0"));
  if (n_alpha < 1 || n_alpha > 8 || !alphas) return finish(ctx, fail(FLSQ_EINVAL, "n_alpha = %d outside [1, 8]", n_alpha));
  const int d = basis->d, n = basis->n_feat;
  uint32_t mask = 0;
  for (int a = 0; a < n_alpha; ++a) {
    int ord = 0;
    for (int k = 0; k < d; ++k) ord += alphas[a * d + k];
    if (ord & 1) mask |= 1u << a;
  }
  const size_t need = eval_scratch_bytes(d, n, n_alpha);
  unsigned char* base = nullptr;
  if (no_alloc) {
    if (need > (size_t)FLSQ_EVAL_SCRATCH_BYTES)
      return finish(ctx, fail(FLSQ_EINVAL,
                              "evaluate_noalloc: d = %d, n_feat = %d, n_alpha = %d need %zu bytes of scratch, above "
                              "the static %d",
                              d, n, n_alpha, need, (int)FLSQ_EVAL_SCRATCH_BYTES));
    if (!ctx->scratch) return finish(ctx, fail(FLSQ_EHIP, "evaluate_noalloc: no scratch address for this device"));
    base = ctx->scratch;
  } else {
    e = ws_get(ctx, "ev_scratch", need, &base);
    if (e.st != FLSQ_OK) return finish(ctx, e);
  }
  const EvalScratch sc = carve_eval(base, d, n, n_alpha);
  hipError_t he = hipMemcpyAsync(sc.al, alphas, (size_t)n_alpha * d, hipMemcpyHostToDevice, ctx->stream);
  if (he == hipSuccess) he = launch_transpose(basis->W, n, d, sc.Wt, nullptr, n, ctx->stream);
  EvalArgs a;
  a.d = d;
  a.n = n;
  a.n_alpha = n_alpha;
  a.n_q = n_q;
  a.Wt = sc.Wt;
  a.b = basis->b;
  a.beta = beta;
  a.alphas = sc.al;
  a.xq = xq;
  a.out = out;
  a.fp32 = xq_is_fp32 ? 1 : 0;
  a.norm = basis->normalize ? 1.0 / std::sqrt((double)n) : 1.0;
  a.coef = sc.coef;
  a.coef32 = sc.coef32;
  a.Wt32 = sc.Wt32;
  a.b32 = sc.b32;
  a.cos_mask = mask;
  if (he == hipSuccess) he = launch_evaluate(a, ctx->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "evaluate: %s", hipGetErrorString(he)));
  return finish(ctx, ok());
}

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================
extern "C" {

flsq_status flsq_create(flsq_ctx** ctx, int device, void* hip_stream) {
  if (!ctx) return FLSQ_EINVAL;
  *ctx = nullptr;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev == 0) return FLSQ_EHIP;
  if (device < 0 || device >= n_dev) return FLSQ_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return FLSQ_EHIP;
  flsq_ctx* c = new flsq_ctx();
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->n_cu = prop.multiProcessorCount;
  if (hipEventCreate(&c->ev0) != hipSuccess || hipEventCreate(&c->ev1) != hipSuccess ||
      hipEventCreate(&c->ev_g0) != hipSuccess || hipEventCreate(&c->ev_g1) != hipSuccess ||
      scratch_address(device, &c->scratch) != hipSuccess) {
    for (hipEvent_t e : {c->ev0, c->ev1, c->ev_g0, c->ev_g1})
      if (e) (void)hipEventDestroy(e);
    delete c;
    return FLSQ_EHIP;
  }
  *ctx = c;
  return FLSQ_OK;
}

void flsq_destroy(flsq_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  for (hipEvent_t e : {ctx->ev0, ctx->ev1, ctx->ev_g0, ctx->ev_g1})
    if (e) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  if (ctx->up) (void)hipHostFree(ctx->up);
  delete ctx->aux_factor;
  delete ctx;
}

const char* flsq_last_error(const flsq_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

const char* flsq_build_info(void) { return "libfastlsq 0.1 (HIP, gfx950)"; }

flsq_status flsq_assemble(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                          int32_t fp32, void* A_out, double* rhs_out) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!A_out) return finish(ctx, fail(FLSQ_EINVAL, "A_out is NULL"));
  Err e = build_system(ctx, ctx->sys, basis, blocks, n_blocks, rhs_out != nullptr);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  const System& s = ctx->sys;
  hipError_t he = launch_assemble(s.geo(), fp32 ? 1 : 0, A_out, ctx->stream);
  if (he == hipSuccess && rhs_out)
    he = hipMemcpyAsync(rhs_out, s.rhs_w.p, sizeof(double) * s.P, hipMemcpyDeviceToDevice, ctx->stream);
  if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "assemble: %s", hipGetErrorString(he)));
  return finish(ctx, ok());
}

flsq_status flsq_gram(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks, int32_t prec,
                      double* G_out, double* c_out) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!G_out) return finish(ctx, fail(FLSQ_EINVAL, "G_out is NULL"));
  SolveParams sp;
  sp.prec = prec;
  Err e = check_params(sp);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  e = build_system(ctx, ctx->sys, basis, blocks, n_blocks, c_out != nullptr);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  const System& s = ctx->sys;
  e = run_gram(ctx, s, prec, nullptr, G_out, 1, 0.0);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (c_out) {
    double* colwork;
    e = ws_get(ctx, "colwork0", pass_work_elems(s.n, s.n_runs, 1) + 64, &colwork);
    if (e.st != FLSQ_OK) return finish(ctx, e);
    hipError_t he = launch_colpass_runs(s.pass(), nullptr, s.rhs_w.as<double>(), 1, nullptr, 1.0, 0.0, c_out, colwork,
                                        ctx->stream);
    if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "colpass: %s", hipGetErrorString(he)));
  }
  hipError_t he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "gram: %s", hipGetErrorString(he)));
  return finish(ctx, ok());
}

flsq_status flsq_solve_linear(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                              const flsq_solve_opts* opts, double* beta_out, flsq_solve_info* info) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!beta_out) return finish(ctx, fail(FLSQ_EINVAL, "beta_out is NULL"));
  const double t0 = now_ms();
  SolveParams sp = params_of(opts);
  Err e = check_params(sp);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (info) memset(info, 0, sizeof *info);
  e = build_system(ctx, ctx->sys, basis, blocks, n_blocks, true);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  bool conv = true;
  e = solve_on_system(ctx, ctx->sys, nullptr, sp, ctx->sys.rhs_w.as<double>(), 1, beta_out, info, &conv);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  e = check_finite_dev(ctx, beta_out, ctx->sys.n, "beta");
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (info) info->t_total_ms = now_ms() - t0;
  if (!conv && sp.refine_tol > 0.0)
    return finish(ctx, fail(FLSQ_ENOCONV, "refinement did not reach refine_tol in %d iterations", sp.max_refine));
  return finish(ctx, ok());
}

flsq_status flsq_factorize(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                           const flsq_solve_opts* opts, flsq_factor** F, flsq_solve_info* info) {
  if (!ctx || !F) return FLSQ_EINVAL;
  *F = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  SolveParams sp = params_of(opts);
  Err e = check_params(sp);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (info) memset(info, 0, sizeof *info);
  flsq_factor* f = new flsq_factor();
  e = factor_into(ctx, f, basis, blocks, n_blocks, sp, info);
  if (e.st != FLSQ_OK) {
    delete f;
    return finish(ctx, e);
  }
  *F = f;
  return finish(ctx, ok());
}

void flsq_factor_free(flsq_factor* F) {
  if (!F) return;
  (void)hipSetDevice(F->device);
  delete F;
}

flsq_status flsq_factor_shape(const flsq_factor* F, int64_t* n_rows, int32_t* n_feat) {
  if (!F) return FLSQ_EINVAL;
  if (n_rows) *n_rows = F->sys.P;
  if (n_feat) *n_feat = F->sys.n;
  return FLSQ_OK;
}

flsq_status flsq_factor_solve(flsq_ctx* ctx, const flsq_factor* F, const double* rhs_rows, int32_t K,
                              double* beta_out, flsq_solve_info* info) {
  if (!ctx || !F) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!rhs_rows || !beta_out) return finish(ctx, fail(FLSQ_EINVAL, "NULL rhs_rows or beta_out"));
  if (K < 1 || K > 64) return finish(ctx, fail(FLSQ_EINVAL, "K = %d outside [1, 64]", K));
  if (info) memset(info, 0, sizeof *info);
  const double t0 = now_ms();
  const System& s = F->sys;
  double* cvec;
  Err e = ws_get(ctx, "cvec", (size_t)s.n * K, &cvec);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  const FactorOp fop(F);
  const LsqOp& op = fop.for_k(K);
  e = op.applyT(ctx, rhs_rows, K, nullptr, 1.0, 0.0, cvec);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  e = chol_solve(ctx, F->Xinv.as<double>(), s.n, cvec, beta_out, K);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  RefineOut ro;
  e = cgls_refine_op(ctx, op, F->Xinv.as<double>(), F->mu, rhs_rows, K, beta_out, F->max_refine, F->refine_tol,
                     info != nullptr, info != nullptr && F->report_grad, &ro);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  hipError_t he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "factor_solve: %s", hipGetErrorString(he)));
  if (info) {
    info->refine_iters = ro.iters;
    info->grad_norm0 = ro.grad0;
    info->grad_norm = ro.grad;
    info->last_step_rel = ro.last_step;
    info->shift = F->shift;
    info->t_total_ms = now_ms() - t0;
  }
  return finish(ctx, ok());
}

flsq_status flsq_factor_solve_normal(flsq_ctx* ctx, const flsq_factor* F, const double* V, int32_t K, double* out) {
  if (!ctx || !F) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!V || !out) return finish(ctx, fail(FLSQ_EINVAL, "NULL V or out"));
  if (K < 1 || K > 64) return finish(ctx, fail(FLSQ_EINVAL, "K = %d outside [1, 64]", K));
  const System& s = F->sys;
  const int n = s.n;
  hipStream_t st = ctx->stream;
  // preconditioned CG on (A^T A + mu I) X = V with the factor's FP64 operator
  double *r, *z, *p, *ap, *tP, *dots, *dwork;
  Err e = ok();
  if (e.st == FLSQ_OK) e = ws_get(ctx, "pcg_r", (size_t)n * K, &r);
  if (e.st == FLSQ_OK) e = ws_get(ctx, "pcg_z", (size_t)n * K, &z);
  if (e.st == FLSQ_OK) e = ws_get(ctx, "pcg_p", (size_t)n * K, &p);
  if (e.st == FLSQ_OK) e = ws_get(ctx, "pcg_ap", (size_t)n * K, &ap);
  if (e.st == FLSQ_OK) e = ws_get(ctx, "pcg_tp", (size_t)s.P * K, &tP);
  if (e.st == FLSQ_OK) e = ws_get(ctx, "pcg_dots", (size_t)10 * K, &dots);
  if (e.st == FLSQ_OK) e = ws_get(ctx, "pcg_dwork", (size_t)512 * K + 64, &dwork);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  const FactorOp fop(F);
  const LsqOp& op = fop.for_k(K);
  auto apply_normal = [&](const double* x, double* y) -> Err {   // y = A^T A x + mu x
    CHECK_ERR(op.apply(ctx, x, K, nullptr, 1.0, 0.0, tP, nullptr));
    CHECK_ERR(op.applyT(ctx, tP, K, x, 1.0, F->mu, y));
    return ok();
  };
  auto body = [&]() -> Err {
    CHECK_ERR(chol_solve(ctx, F->Xinv.as<double>(), n, V, out, K));
    if (F->max_refine == 0) return ok();
    std::vector<double> tmp;
    CHECK_ERR(apply_normal(out, ap));
    CHECK_HIP(hipMemcpyAsync(r, V, sizeof(double) * n * K, hipMemcpyDeviceToDevice, st));
    std::vector<double> ones(K, 1.0);
    CHECK_HIP(launch_axpy_cols(cols(ones), ap, r, n, K, -1.0, st));
    // Per-column scalars stay on the device: gam | alpha | (unused) | p.Mp | x.V before the step |
    // x.V | x.r | gam_new (gam and gam_new alternate); the host reads them once per iteration.
    double* d_gam = dots;
    double *d_alpha = dots + K, *d_pap = dots + 3 * K, *d_xv0 = dots + 4 * K;
    double *d_xv = dots + 5 * K, *d_xr = dots + 6 * K, *d_gnew = dots + 7 * K;
    CHECK_ERR(chol_solve(ctx, F->Xinv.as<double>(), n, r, z, K));
    CHECK_HIP(launch_cg_direction(r, z, p, n, K, nullptr, d_gam, dwork, st));   // gam = r.z, p = z
    // Stop when the step's energy norm |alpha| (p^T M p)^{1/2} (M = G + mu I) is below tol
    // times the solution's, estimated by (out^T V)^{1/2}.  The energy functional
    // phi(x) = x^T M x / 2 - x^T V = -(x^T V + x^T r) / 2 decreases monotonically in exact
    // arithmetic; a column whose phi clearly rises stops, and its last iterate before the
    // rise is returned.
    double* xbest;
    CHECK_ERR(ws_get(ctx, "pcg_xbest", (size_t)n * K, &xbest));
    CHECK_HIP(hipMemcpyAsync(xbest, out, sizeof(double) * n * K, hipMemcpyDeviceToDevice, st));
    {
      DotBatch db{};
      db.K = K;
      db.count = 2;
      db.x[0] = db.x[1] = out;
      db.y[0] = V;
      db.y[1] = r;
      db.n[0] = db.n[1] = n;
      db.out[0] = d_xv;
      db.out[1] = d_xr;
      CHECK_HIP(launch_dot_batch(db, dwork, st));
    }
    CHECK_ERR(host_cols(ctx, d_xv, 2 * K, tmp));
    std::vector<double> phibest(K), active(K, 1.0), improved(K, 0.0), relstep(K, 0.0), minstep(K, HUGE_VAL);
    std::vector<int> stagnant(K, 0);
    for (int k = 0; k < K; ++k) phibest[k] = -0.5 * (tmp[k] + tmp[K + k]);
    std::vector<double> hs(6 * K);
    uint64_t keep_mask = 0;
    for (int it = 0; it < F->max_refine; ++it) {
      CHECK_ERR(apply_normal(p, ap));
      {
        DotBatch db{};
        db.K = K;
        db.count = 2;
        db.x[0] = p;
        db.y[0] = ap;
        db.n[0] = n;
        db.out[0] = d_pap;
        db.x[1] = out;
        db.y[1] = V;
        db.n[1] = n;
        db.out[1] = d_xv0;
        CHECK_HIP(launch_dot_batch(db, dwork, st));
      }
      {
        AxpyBatch ab{};
        ab.K = K;
        ab.count = 2;
        ab.x[0] = p;
        ab.y[0] = out;
        ab.n[0] = n;
        ab.sign[0] = 1.0;
        ab.x[1] = ap;
        ab.y[1] = r;
        ab.n[1] = n;
        ab.sign[1] = -1.0;
        CHECK_HIP(launch_cg_step(d_gam, d_pap, nullptr, 0.0, col_mask(active), d_alpha, ab, xbest, keep_mask, st));
        keep_mask = 0;
      }
      {
        DotBatch db{};
        db.K = K;
        db.count = 2;
        db.x[0] = out;
        db.y[0] = V;
        db.n[0] = n;
        db.out[0] = d_xv;
        db.x[1] = out;
        db.y[1] = r;
        db.n[1] = n;
        db.out[1] = d_xr;
        CHECK_HIP(launch_dot_batch(db, dwork, st));
      }
      CHECK_ERR(read_back(ctx, hs.data(), d_alpha, sizeof(double) * 6 * K));
      const double *h_alpha = hs.data(), *h_pap = hs.data() + 2 * K, *h_xv0 = hs.data() + 3 * K;
      const double *h_xv = hs.data() + 4 * K, *h_xr = hs.data() + 5 * K;
      double worst = 0.0;
      for (int k = 0; k < K; ++k) {
        if (active[k] > 0.0) {
          const double prev = relstep[k];
          relstep[k] = std::fabs(h_alpha[k]) * std::sqrt(std::max(h_pap[k], 0.0)) /
                       std::max(std::sqrt(std::fabs(h_xv0[k])), 1e-300);
          worst = std::max(worst, predicted_step(it, prev, relstep[k]));
        }
      }
      // A column is done once, for two iterations in a row, neither its energy phi dropped
      // by more than a few units in the last place nor its step shrank below half the
      // smallest so far: FP64 no longer resolves its progress (phi is quadratic in the error
      // and stops resolving it long before the step does).  phi is formed from dot products
      // whose terms cancel (x^T V is far smaller than |x|^T |V|), so its rounding noise can
      // reach 1e-12 relative while the error still falls by orders of magnitude: only a rise
      // above sqrt(eps) relative (an energy-norm error near 1e-4), far above that noise,
      // counts as divergence.
      int n_active = 0;
      const double rise = std::sqrt(DBL_EPSILON);
      for (int k = 0; k < K; ++k) {
        improved[k] = 0.0;
        if (active[k] == 0.0) continue;
        const double phi = -0.5 * (h_xv[k] + h_xr[k]);
        const bool resolved =
            (phibest[k] - phi) > 4.0 * DBL_EPSILON * std::fabs(phibest[k]) || relstep[k] < 0.5 * minstep[k];
        minstep[k] = std::min(minstep[k], relstep[k]);
        if (phi <= phibest[k] + rise * std::fabs(phibest[k])) {
          phibest[k] = std::min(phibest[k], phi);
          improved[k] = 1.0;
        } else {
          active[k] = 0.0;
        }
        stagnant[k] = resolved ? 0 : stagnant[k] + 1;
        if (stagnant[k] >= 2) active[k] = 0.0;
        if (active[k] > 0.0) ++n_active;
      }
      keep_mask = col_mask(improved);   // copied by the next step's launch, or below
      if (worst <= F->refine_tol || n_active == 0 || it + 1 == F->max_refine) break;
      CHECK_ERR(chol_solve(ctx, F->Xinv.as<double>(), n, r, z, K));
      CHECK_HIP(launch_cg_direction(r, z, p, n, K, d_gam, d_gnew, dwork, st));
      std::swap(d_gam, d_gnew);
    }
    if (keep_mask) CHECK_HIP(launch_select_cols(out, xbest, n, K, keep_mask, st));
    CHECK_HIP(hipMemcpyAsync(out, xbest, sizeof(double) * n * K, hipMemcpyDeviceToDevice, st));
    return ok();
  };
  e = body();
  if (e.st != FLSQ_OK) return finish(ctx, e);
  hipError_t he = hipStreamSynchronize(st);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "solve_normal: %s", hipGetErrorString(he)));
  return finish(ctx, ok());
}

flsq_status flsq_apply_A(flsq_ctx* ctx, const flsq_factor* F, const double* V, int32_t K, double* out) {
  if (!ctx || !F) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!V || !out) return finish(ctx, fail(FLSQ_EINVAL, "NULL V or out"));
  if (K < 1 || K > 64) return finish(ctx, fail(FLSQ_EINVAL, "K = %d outside [1, 64]", K));
  const FactorOp fop(F);
  Err e = fop.for_k(K).apply(ctx, V, K, nullptr, 1.0, 0.0, out, nullptr);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  hipError_t he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "apply_A: %s", hipGetErrorString(he)));
  return finish(ctx, ok());
}

flsq_status flsq_apply_At(flsq_ctx* ctx, const flsq_factor* F, const double* Y, int32_t K, double* out) {
  if (!ctx || !F) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!Y || !out) return finish(ctx, fail(FLSQ_EINVAL, "NULL Y or out"));
  if (K < 1 || K > 64) return finish(ctx, fail(FLSQ_EINVAL, "K = %d outside [1, 64]", K));
  const FactorOp fop(F);
  Err e = fop.for_k(K).applyT(ctx, Y, K, nullptr, 1.0, 0.0, out);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  hipError_t he = hipStreamSynchronize(ctx->stream);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "apply_At: %s", hipGetErrorString(he)));
  return finish(ctx, ok());
}

flsq_status flsq_evaluate(flsq_ctx* ctx, const flsq_basis* basis, const double* beta, int64_t n_q, const void* xq,
                          int32_t xq_is_fp32, const uint8_t* alphas, int32_t n_alpha, void* out) {
  return evaluate_entry(ctx, basis, beta, n_q, xq, xq_is_fp32, alphas, n_alpha, out, false);
}

flsq_status flsq_evaluate_noalloc(flsq_ctx* ctx, const flsq_basis* basis, const double* beta, int64_t n_q,
                                  const void* xq, int32_t xq_is_fp32, const uint8_t* alphas, int32_t n_alpha,
                                  void* out) {
  return evaluate_entry(ctx, basis, beta, n_q, xq, xq_is_fp32, alphas, n_alpha, out, true);
}

}  // extern "C"

// =====================================================================================
// Newton-Raphson (Section 2.4)
// =====================================================================================
namespace {

Err newton_impl(flsq_ctx* c, const flsq_basis* basis, const flsq_rows* blocks, int n_blocks, int nl_block,
                const flsq_nonlin* nl, const flsq_newton_opts* o, double* beta, flsq_newton_trace* tr,
                bool* converged) {
  if (!nl || nl->n_poly < 1 || nl->n_poly > 16 || !nl->poly) return fail(FLSQ_EINVAL, "nonlinearity: n_poly in [1, 16]");
  if (!o) return fail(FLSQ_EINVAL, "opts is NULL");
  if (o->max_iter < 0 || o->max_iter > 64) return fail(FLSQ_EINVAL, "max_iter outside [0, 64]");
  if (o->max_halvings < 0 || o->max_halvings > 60) return fail(FLSQ_EINVAL, "max_halvings outside [0, 60]");
  if (!(o->armijo_c >= 0.0 && o->armijo_c < 1.0)) return fail(FLSQ_EINVAL, "armijo_c outside [0, 1)");
  if (o->refactor_iters < 0) return fail(FLSQ_EINVAL, "refactor_iters must be >= 0");
  if (!beta) return fail(FLSQ_EINVAL, "beta_inout is NULL");
  SolveParams sp = params_of(&o->lin);
  CHECK_ERR(check_params(sp));
  System& s = c->sys;
  CHECK_ERR(build_system(c, s, basis, blocks, n_blocks, true));
  if (nl_block < 0 || nl_block >= n_blocks) return fail(FLSQ_EINVAL, "nonlin_block %d outside [0, %d)", nl_block, n_blocks);
  if (!s.even[nl_block])
    return fail(FLSQ_EINVAL, "the nonlinear block's operator must have even-order terms only");
  for (int k = 0; k < nl->n_poly; ++k)
    if (!std::isfinite(nl->poly[k])) return fail(FLSQ_ENONFINITE, "nonlinearity coefficient not finite");
  const int n = s.n;
  const int64_t P = s.P;
  hipStream_t st = c->stream;
  double *poly, *R, *Rt, *rho, *rhot, *u, *ut, *delta, *bt, *negR, *dots, *dwork;
  CHECK_ERR(ws_get(c, "nt_poly", 16, &poly));
  CHECK_ERR(ws_get(c, "nt_R", (size_t)P, &R));
  CHECK_ERR(ws_get(c, "nt_Rt", (size_t)P, &Rt));
  CHECK_ERR(ws_get(c, "nt_rho", (size_t)P, &rho));
  CHECK_ERR(ws_get(c, "nt_rhot", (size_t)P, &rhot));
  CHECK_ERR(ws_get(c, "nt_u", (size_t)P, &u));
  CHECK_ERR(ws_get(c, "nt_ut", (size_t)P, &ut));
  CHECK_ERR(ws_get(c, "nt_delta", (size_t)n, &delta));
  CHECK_ERR(ws_get(c, "nt_bt", (size_t)n, &bt));
  CHECK_ERR(ws_get(c, "nt_negR", (size_t)P, &negR));
  CHECK_ERR(ws_get(c, "nt_dots", 8, &dots));
  CHECK_ERR(ws_get(c, "nt_dwork", 1024, &dwork));
  CHECK_HIP(hipMemcpyAsync(poly, nl->poly, sizeof(double) * nl->n_poly, hipMemcpyHostToDevice, st));
  const double w_nl = s.weight[nl_block];
  const int64_t nl0 = s.row0[nl_block], nln = s.rows[nl_block];
  const PassGeo pg = s.pass();
  double* rpwork = nullptr;
  if (const size_t we = rowpass_work_elems(pg, 1)) CHECK_ERR(ws_get(c, "nt_rpwork", we, &rpwork));
  auto residual = [&](const double* b, double* Rout, double* rho_out, double* u_out, double* nrm) -> Err {
    CHECK_HIP(launch_newton_residual_runs(pg, b, s.rhs_w.as<double>(), nl_block, poly, nl->n_poly, w_nl, s.norm, Rout,
                                          rho_out, u_out, rpwork, st));
    CHECK_HIP(launch_dot_cols(Rout, Rout, P, 1, dots, dwork, st));
    double h = 0.0;
    CHECK_ERR(read_back(c, &h, dots, sizeof(double)));
    *nrm = std::sqrt(h);
    if (!std::isfinite(*nrm)) return fail(FLSQ_ENONFINITE, "Newton residual is not finite");
    return ok();
  };
  auto dot1 = [&](const double* x, const double* y, int64_t len, double* out) -> Err {
    CHECK_HIP(launch_dot_cols(x, y, len, 1, dots, dwork, st));
    CHECK_ERR(read_back(c, out, dots, sizeof(double)));
    return ok();
  };
  const double t0 = now_ms();
  // The Gram changes little between steps, so a shift that made the factor positive
  // definite is kept as the starting shift of the next factorisation (no repeated retries).
  SolveParams spk = sp;
  flsq_solve_info sinfo;
  // The factor held in Xinv: the warm start's (the linear operator's Gram), then that of the
  // last step that formed its own.  Its shift is reported for the steps it preconditions.
  bool have_factor = false;
  double held_shift = 0.0;
  if (o->warm_start) {
    // linear part only: the nonlinearity dropped, rho = 0
    CHECK_ERR(solve_on_system(c, s, nullptr, spk, s.rhs_w.as<double>(), 1, beta, &sinfo, nullptr));
    spk.shift_rel = std::max(spk.shift_rel, sinfo.shift);
    have_factor = true;
    held_shift = sinfo.shift;
  }
  // Newton steps need no fully refined step: the automatic second pass is left to the warm
  // start (measured: on the reaction-diffusion steps it costs more than the CG steps it saves)
  if (spk.second_pass == 0) spk.second_pass = -1;
  if (tr) memset(tr, 0, sizeof *tr);
  *converged = false;
  double nR = 0.0;
  CHECK_ERR(residual(beta, R, rho, u, &nR));
  std::vector<double> one(1, 1.0);
  for (int it = 0; it < o->max_iter; ++it) {
    // delta = argmin ||J delta + R||^2 + mu ||delta||^2 with J = A(rho)
    CHECK_HIP(launch_scale_copy(R, negR, P, -1.0, st));
    const double ts = now_ms();
    bool factored = true;
    if (o->refactor_iters > 0 && have_factor) {
      CHECK_ERR(solve_reusing_factor(c, s, rho, spk, negR, 1, delta, o->refactor_iters, &sinfo, nullptr, &factored));
    } else {
      CHECK_ERR(solve_on_system(c, s, rho, spk, negR, 1, delta, &sinfo, nullptr));
    }
    const double t_solve = now_ms() - ts;
    if (factored) {
      spk.shift_rel = std::max(spk.shift_rel, sinfo.shift);
      held_shift = sinfo.shift;
      have_factor = true;
    }
    double alpha = 1.0, nRt = 0.0;
    int halv = 0;
    for (;;) {
      CHECK_HIP(hipMemcpyAsync(bt, beta, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      one[0] = alpha;
      CHECK_HIP(launch_axpy_cols(cols(one), delta, bt, n, 1, 1.0, st));
      CHECK_ERR(residual(bt, Rt, rhot, ut, &nRt));
      if (nRt <= (1.0 - o->armijo_c * alpha) * nR || halv >= o->max_halvings) break;
      alpha *= 0.5;
      ++halv;
    }
    double dd = 0.0, du2 = 0.0, un2 = 0.0;
    CHECK_ERR(dot1(delta, delta, n, &dd));
    const double step = alpha * std::sqrt(dd);
    // ||Delta u|| / ||u|| on the rows of the nonlinear block
    CHECK_HIP(hipMemcpyAsync(negR, ut + nl0, sizeof(double) * nln, hipMemcpyDeviceToDevice, st));
    one[0] = 1.0;
    CHECK_HIP(launch_axpy_cols(cols(one), u + nl0, negR, nln, 1, -1.0, st));
    CHECK_ERR(dot1(negR, negR, nln, &du2));
    CHECK_ERR(dot1(ut + nl0, ut + nl0, nln, &un2));
    if (tr) {
      tr->res_norm[it] = nR;
      tr->alpha[it] = alpha;
      tr->halvings[it] = halv;
      tr->step_norm[it] = step;
      tr->du_rel[it] = std::sqrt(du2) / std::max(std::sqrt(un2), 1e-300);
      tr->refine_iters[it] = sinfo.refine_iters;
      tr->shift[it] = held_shift;
      tr->t_solve_ms[it] = t_solve;
      tr->factored[it] = factored ? 1 : 0;
      tr->iters = it + 1;
    }
    CHECK_HIP(hipMemcpyAsync(beta, bt, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    std::swap(R, Rt);
    std::swap(rho, rhot);
    std::swap(u, ut);
    nR = nRt;
    if (step < o->tol_dbeta) {
      *converged = true;
      break;
    }
  }
  CHECK_HIP(hipStreamSynchronize(st));
  if (tr) {
    tr->converged = *converged ? 1 : 0;
    tr->t_total_ms = now_ms() - t0;
  }
  return check_finite_dev(c, beta, n, "beta");
}

// Derived geometry on the rows of a factor: same features, another operator / row set.
Err build_rows_on(flsq_ctx* c, System& out, const System& base, const double* x_rowmajor, int64_t rows,
                  const flsq_term* terms, int n_terms, double weight) {
  flsq_basis bs;
  bs.d = base.d;
  bs.n_feat = base.n;
  bs.W = base.Wrm.as<double>();
  bs.b = base.bvec.as<double>();
  bs.normalize = base.normalize;
  flsq_rows r;
  r.n_rows = rows;
  r.x = x_rowmajor;
  r.op.terms = terms;
  r.op.n_terms = n_terms;
  r.weight = weight;
  r.rhs = nullptr;
  return build_system(c, out, &bs, &r, 1, false);
}

Err inverse_impl(flsq_ctx* c, flsq_factor* F, int64_t n_src, double src_weight, int n_lap, const double* thetas, int K,
                 int64_t n_obs, const double* x_obs, const double* data, double* loss, double* gtheta,
                 double* gkappa) {
  const System& s = F->sys;
  if (K < 1 || K > 64) return fail(FLSQ_EINVAL, "K = %d outside [1, 64]", K);
  if (n_src < 1 || n_src > s.P) return fail(FLSQ_EINVAL, "n_src_rows outside [1, P]");
  if (s.d < 2) return fail(FLSQ_EINVAL, "the source needs two spatial coordinates");
  if (n_lap < 0 || n_lap > s.d) return fail(FLSQ_EINVAL, "n_lap_dims outside [0, d]");
  if (n_obs < 1 || !x_obs || !data || !thetas || !loss || !gtheta) return fail(FLSQ_EINVAL, "NULL argument");
  hipStream_t st = c->stream;
  const int n = s.n;
  const int64_t P = s.P;
  // observation rows H (identity operator) and the interior dA/dkappa rows, cached on the factor
  flsq_term ident;
  memset(&ident, 0, sizeof ident);
  ident.coef = 1.0;
  if (F->obs_key != (const void*)x_obs || F->obs_n != n_obs) {
    CHECK_ERR(build_rows_on(c, F->obs, s, x_obs, n_obs, &ident, 1, 1.0));
    F->obs_key = x_obs;
    F->obs_n = n_obs;
  }
  if (gkappa && (F->akap_rows != n_src || F->akap_dims != n_lap || F->akap_weight != src_weight)) {
    // interior operator d/dt - kappa sum_k D^{2 e_k}: dA/dkappa = -sum_{k < n_lap} D^{2 e_k}
    flsq_term t[FLSQ_MAX_DIM];
    memset(t, 0, sizeof t);
    for (int k = 0; k < n_lap; ++k) {
      t[k].coef = -1.0;
      t[k].alpha[k] = 2;
    }
    if (n_lap == 0) return fail(FLSQ_EINVAL, "kappa gradient needs n_lap_dims >= 1");
    CHECK_ERR(build_rows_on(c, F->akap, s, s.Xrm.as<double>(), n_src, t, n_lap, src_weight));
    F->akap_rows = n_src;
    F->akap_dims = n_lap;
    F->akap_weight = src_weight;
  }
  double *Rhs, *B, *U, *gu, *Vn, *Lam, *AL, *gwork, *colwork;
  CHECK_ERR(ws_get(c, "inv_rhs", (size_t)P * K, &Rhs));
  CHECK_ERR(ws_get(c, "inv_B", (size_t)n * K, &B));
  CHECK_ERR(ws_get(c, "inv_U", (size_t)n_obs * K, &U));
  CHECK_ERR(ws_get(c, "inv_gu", (size_t)n_obs * K, &gu));
  CHECK_ERR(ws_get(c, "inv_V", (size_t)n * K, &Vn));
  CHECK_ERR(ws_get(c, "inv_lam", (size_t)n * K, &Lam));
  CHECK_ERR(ws_get(c, "inv_AL", (size_t)P * K, &AL));
  CHECK_ERR(ws_get(c, "inv_gwork", (size_t)K * 64 * 4 + 64, &gwork));
  CHECK_ERR(ws_get(c, "inv_colwork", pass_work_elems(n, F->obs.n_runs, K) + 64, &colwork));
  CHECK_HIP(launch_source(s.Xt.as<double>(), P, n_src, src_weight, thetas, K, Rhs, st));
  if (!gkappa && F->rep_key == (const void*)x_obs && F->rep_nobs == n_obs && F->rep_nsrc == n_src) {
    // observation operator kept: U = R rhs_src, (A Lam)_src = R^T (2/n_obs)(U - data)
    double* part = nullptr;
    const size_t we = std::max(gemm_t16_work_elems(n_obs, n_src, K), gemm_t16_work_elems(n_src, n_obs, K));
    if (we) CHECK_ERR(ws_get(c, "inv_t16part", we, &part));
    CHECK_HIP(launch_gemm_t16(F->R16.as<double>(), n_obs, n_src, Rhs, K, nullptr, 1.0, 0.0, U, part, st));
    CHECK_HIP(launch_misfit(U, data, n_obs, K, loss, gu, st));
    CHECK_HIP(launch_gemm_t16(F->Rt16.as<double>(), n_src, n_obs, gu, K, nullptr, 1.0, 0.0, AL, part, st));
    CHECK_HIP(launch_source_grad_dot(s.Xt.as<double>(), P, n_src, src_weight, thetas, K, AL, gtheta, gwork, st));
    CHECK_HIP(hipStreamSynchronize(st));
    return ok();
  }
  // forward: B = (A^T A + mu I)^{-1} A^T rhs(theta), U = H B, misfit
  flsq_status fs = flsq_factor_solve(c, F, Rhs, K, B, nullptr);
  if (fs != FLSQ_OK) return Err{fs, c->err};
  CHECK_ERR(row_pass(c, F->obs.pass(), nullptr, B, K, nullptr, 1.0, 0.0, U));
  CHECK_HIP(launch_misfit(U, data, n_obs, K, loss, gu, st));
  // backward: Lam = (A^T A + mu I)^{-1} H^T gu ; AL = A Lam ; dL/dtheta = AL^T d rhs / d theta
  CHECK_HIP(launch_colpass_runs(F->obs.pass(), nullptr, gu, K, nullptr, 1.0, 0.0, Vn, colwork, st));
  fs = flsq_factor_solve_normal(c, F, Vn, K, Lam);
  if (fs != FLSQ_OK) return Err{fs, c->err};
  const FactorOp fop(F);
  const LsqOp& op = fop.for_k(K);
  CHECK_ERR(op.apply(c, Lam, K, nullptr, 1.0, 0.0, AL, nullptr));
  CHECK_HIP(launch_source_grad_dot(s.Xt.as<double>(), P, n_src, src_weight, thetas, K, AL, gtheta, gwork, st));
  if (gkappa) {
    // dL/dkappa = (A_k Lam)^T (rhs - A B) - (A Lam)^T (A_k B), A_k nonzero on the interior rows only
    double *r, *AkL, *AkB, *dots, *dwork;
    CHECK_ERR(ws_get(c, "inv_r", (size_t)P * K, &r));
    CHECK_ERR(ws_get(c, "inv_AkL", (size_t)n_src * K, &AkL));
    CHECK_ERR(ws_get(c, "inv_AkB", (size_t)n_src * K, &AkB));
    CHECK_ERR(ws_get(c, "inv_dots", (size_t)2 * K, &dots));
    CHECK_ERR(ws_get(c, "inv_dwork", (size_t)512 * K + 64, &dwork));
    CHECK_ERR(op.apply(c, B, K, Rhs, -1.0, 1.0, r, nullptr));
    CHECK_ERR(row_pass(c, F->akap.pass(), nullptr, Lam, K, nullptr, 1.0, 0.0, AkL));
    CHECK_ERR(row_pass(c, F->akap.pass(), nullptr, B, K, nullptr, 1.0, 0.0, AkB));
    CHECK_HIP(launch_dot_cols(AkL, r, n_src, K, dots, dwork, st));
    CHECK_HIP(launch_dot_cols(AL, AkB, n_src, K, dots + K, dwork, st));
    CHECK_HIP(launch_combine_diff(dots, dots + K, gkappa, K, st));
  }
  CHECK_HIP(hipStreamSynchronize(st));
  return ok();
}

// R = H (A^T A + mu I)^{-1} A_src^T, built a block of 64 observations at a time: the block's
// rows of H transposed (n x kb), the refined normal-equation solve with the factor, A applied
// to the solutions, and its first n_src rows written into the block's columns of R^T.
Err inverse_prepare_impl(flsq_ctx* c, flsq_factor* F, int64_t n_src, int64_t n_obs, const double* x_obs) {
  const System& s = F->sys;
  if (n_src < 1 || n_src > s.P) return fail(FLSQ_EINVAL, "n_src_rows outside [1, P]");
  if (n_obs < 1 || !x_obs) return fail(FLSQ_EINVAL, "need n_obs >= 1 observation points");
  hipStream_t st = c->stream;
  const int n = s.n;
  const int64_t P = s.P;
  flsq_term ident;
  memset(&ident, 0, sizeof ident);
  ident.coef = 1.0;
  if (F->obs_key != (const void*)x_obs || F->obs_n != n_obs) {
    CHECK_ERR(build_rows_on(c, F->obs, s, x_obs, n_obs, &ident, 1, 1.0));
    F->obs_key = x_obs;
    F->obs_n = n_obs;
  }
  F->rep_key = nullptr;
  double *H, *Hb, *Zb, *AZ, *Rt;
  CHECK_ERR(ws_get(c, "rep_H", (size_t)n_obs * n, &H));
  CHECK_ERR(ws_get(c, "rep_Hb", (size_t)n * 64, &Hb));
  CHECK_ERR(ws_get(c, "rep_Zb", (size_t)n * 64, &Zb));
  CHECK_ERR(ws_get(c, "rep_AZ", (size_t)P * 64, &AZ));
  CHECK_ERR(ws_get(c, "rep_Rt", (size_t)n_src * n_obs, &Rt));
  CHECK_HIP(launch_assemble(F->obs.geo(), 0, H, st));
  const FactorOp fop(F);
  for (int64_t b0 = 0; b0 < n_obs; b0 += 64) {
    const int kb = (int)std::min<int64_t>(64, n_obs - b0);
    CHECK_HIP(launch_transpose_f64(H + b0 * n, kb, n, Hb, st));
    const flsq_status fs = flsq_factor_solve_normal(c, F, Hb, kb, Zb);
    if (fs != FLSQ_OK) return Err{fs, c->err};
    CHECK_ERR(fop.for_k(kb).apply(c, Zb, kb, nullptr, 1.0, 0.0, AZ, nullptr));
    CHECK_HIP(hipMemcpy2DAsync(Rt + b0, sizeof(double) * n_obs, AZ, sizeof(double) * kb, sizeof(double) * kb, n_src,
                               hipMemcpyDeviceToDevice, st));
  }
  if (F->R16.ensure(sizeof(double) * t16_elems(n_obs, n_src)) != hipSuccess ||
      F->Rt16.ensure(sizeof(double) * t16_elems(n_src, n_obs)) != hipSuccess)
    return fail(FLSQ_ENOMEM, "observation operator allocation failed");
  CHECK_HIP(launch_to_t16(Rt, n_obs, n_src, 1, F->R16.as<double>(), st));
  CHECK_HIP(launch_to_t16(Rt, n_src, n_obs, 0, F->Rt16.as<double>(), st));
  CHECK_HIP(hipStreamSynchronize(st));
  F->rep_key = x_obs;
  F->rep_nobs = n_obs;
  F->rep_nsrc = n_src;
  return ok();
}

// Learnable bandwidth (the paper's reparameterisation appendix): W_j = L What_j, outer loss
// Lo = ||A beta* - b||^2 at the Tikhonov solution.  With r = b - A beta*, M = A^T A + mu I,
// lam = M^{-1} beta* and A' = dA/dL_pq (using A^T r = mu beta*):
//   dLo/dL_pq = -2 [r^T A' beta* + mu (r^T A' lam - (A lam)^T A' beta*)].
// dA_ij/dL_pq = What_jq dA_ij/dW_jp, and from Eq. (2)
//   d/dW_jp [W^a Phi_|a|(z)] = a_p W^(a - e_p) Phi_|a|(z) + W^a Phi_|a|+1(z) x_ip,
// two operators in the folded form with a quarter-period phase shift (Phi_{k+1}(z) =
// Phi_k(z + pi/2)): T1_p with terms (c a_p, a - e_p), and T2 = the operator itself; the x_ip
// factor weights the rows and What_jq the feature vector, so every form is a row pass.
Err shift_phase(flsq_ctx* c, System& s, double delta) {
  CHECK_HIP(launch_add_phase(s.ph.as<double>(), (int64_t)s.n_blocks * s.n, delta, c->stream));
  CHECK_HIP(launch_pack_features(s.Wrm.as<double>(), s.amp.as<double>(), s.ph.as<double>(), s.n_blocks, s.n, s.d,
                                 s.frec.as<double>(), c->stream));
  return ok();
}

Err bandwidth_impl(flsq_ctx* c, const flsq_basis* base, const double* L, const flsq_rows* blocks, int n_blocks,
                   const flsq_solve_opts* opts, double* beta, double* loss_out, double* grad_out) {
  CHECK_ERR(check_basis(base));
  if (!L || !beta || !loss_out || !grad_out || !opts) return fail(FLSQ_EINVAL, "NULL argument");
  if (!blocks || n_blocks < 1) return fail(FLSQ_EINVAL, "need at least one row block");
  for (int i = 0; i < n_blocks; ++i)
    if (!blocks[i].rhs && blocks[i].n_rows > 0) return fail(FLSQ_EINVAL, "block %d has no data (rhs)", i);
  const int d = base->d, n = base->n_feat;
  for (int p = 0; p < d; ++p)
    for (int q = 0; q < d; ++q) {
      if (!std::isfinite(L[p * d + q])) return fail(FLSQ_ENONFINITE, "L is not finite");
      if (q > p && L[p * d + q] != 0.0) return fail(FLSQ_EINVAL, "L must be lower triangular");
    }
  hipStream_t st = c->stream;
  double* W;
  CHECK_ERR(ws_get(c, "bw_W", (size_t)n * d, &W));
  LowerMat Lm{};
  for (int p = 0; p < d; ++p)
    for (int q = 0; q <= p; ++q) Lm.v[p * kMaxDim + q] = L[p * d + q];
  CHECK_HIP(launch_apply_lower(base->W, n, d, Lm, W, st));
  flsq_basis bs = *base;
  bs.W = W;
  SolveParams sp = params_of(opts);
  CHECK_ERR(check_params(sp));
  if (!c->aux_factor) c->aux_factor = new flsq_factor();
  flsq_factor* F = c->aux_factor;
  CHECK_ERR(factor_into(c, F, &bs, blocks, n_blocks, sp, nullptr));
  flsq_status fs;
  const System& s = F->sys;
  const int64_t P = s.P;
  const int K = 2 * d;
  fs = flsq_factor_solve(c, F, s.rhs_w.as<double>(), 1, beta, nullptr);
  if (fs != FLSQ_OK) return Err{fs, c->err};
  double *r, *lam, *Alam, *V, *Y, *sums, *work;
  CHECK_ERR(ws_get(c, "bw_r", (size_t)P, &r));
  CHECK_ERR(ws_get(c, "bw_lam", (size_t)n, &lam));
  CHECK_ERR(ws_get(c, "bw_alam", (size_t)P, &Alam));
  CHECK_ERR(ws_get(c, "bw_V", (size_t)n * K, &V));
  CHECK_ERR(ws_get(c, "bw_Y", (size_t)P * K, &Y));
  CHECK_ERR(ws_get(c, "bw_sums", (size_t)2 * K, &sums));
  CHECK_ERR(ws_get(c, "bw_work", (size_t)512 * K + 64, &work));
  // r = b - A beta* and the loss
  CHECK_ERR(row_pass(c, s.pass(), nullptr, beta, 1, s.rhs_w.as<double>(), -1.0, 1.0, r));
  std::vector<double> h;
  CHECK_HIP(launch_dot_cols(r, r, P, 1, sums, work, st));
  CHECK_ERR(host_cols(c, sums, 1, h));
  const double loss = h[0];
  // lam = M^{-1} beta*, A lam, and the feature-scaled vectors [beta* What_q | lam What_q]
  fs = flsq_factor_solve_normal(c, F, beta, 1, lam);
  if (fs != FLSQ_OK) return Err{fs, c->err};
  CHECK_ERR(row_pass(c, s.pass(), nullptr, lam, 1, nullptr, 1.0, 0.0, Alam));
  CHECK_HIP(launch_scaled_cols(beta, lam, base->W, n, d, V, st));
  const double* X = s.Xrm.as<double>();
  const double mu = F->mu;
  // T2: the operator itself, a quarter period on; its forms carry the x_ip row weights
  std::vector<double> s3((size_t)d * K), s4((size_t)d * K);
  {
    System& T2 = c->aux;
    CHECK_ERR(build_system(c, T2, &bs, blocks, n_blocks, false));
    CHECK_ERR(shift_phase(c, T2, 0.5 * M_PI));
    CHECK_ERR(row_pass(c, T2.pass(), nullptr, V, K, nullptr, 1.0, 0.0, Y));
    for (int p = 0; p < d; ++p) {
      CHECK_HIP(launch_wsum_cols(Y, P, K, r, X, d, p, sums, work, st));
      CHECK_HIP(launch_wsum_cols(Y, P, K, Alam, X, d, p, sums + K, work, st));
      CHECK_ERR(host_cols(c, sums, 2 * K, h));
      for (int k = 0; k < K; ++k) {
        s3[(size_t)p * K + k] = h[k];
        s4[(size_t)p * K + k] = h[K + k];
      }
    }
  }
  std::vector<double> grad;
  for (int p = 0; p < d; ++p) {
    // T1_p: terms (c a_p, a - e_p) of every block (a zero term where no alpha has a p component)
    std::vector<std::vector<flsq_term>> terms(n_blocks);
    std::vector<flsq_rows> rows(blocks, blocks + n_blocks);
    for (int i = 0; i < n_blocks; ++i) {
      for (int t = 0; t < blocks[i].op.n_terms; ++t) {
        const flsq_term& tm = blocks[i].op.terms[t];
        if (tm.alpha[p] == 0) continue;
        flsq_term nt = tm;
        nt.coef = tm.coef * tm.alpha[p];
        nt.alpha[p] = (uint8_t)(tm.alpha[p] - 1);
        terms[i].push_back(nt);
      }
      if (terms[i].empty()) {
        flsq_term zt;
        memset(&zt, 0, sizeof zt);
        terms[i].push_back(zt);
      }
      rows[i].op.terms = terms[i].data();
      rows[i].op.n_terms = (int32_t)terms[i].size();
    }
    System& T1 = c->aux;
    CHECK_ERR(build_system(c, T1, &bs, rows.data(), n_blocks, false));
    CHECK_ERR(shift_phase(c, T1, 0.5 * M_PI));
    CHECK_ERR(row_pass(c, T1.pass(), nullptr, V, K, nullptr, 1.0, 0.0, Y));
    CHECK_HIP(launch_wsum_cols(Y, P, K, r, nullptr, 0, 0, sums, work, st));
    CHECK_HIP(launch_wsum_cols(Y, P, K, Alam, nullptr, 0, 0, sums + K, work, st));
    CHECK_ERR(host_cols(c, sums, 2 * K, h));
    for (int q = 0; q <= p; ++q) {
      const double rb = h[q] + s3[(size_t)p * K + q];              // r^T A' beta*
      const double rl = h[d + q] + s3[(size_t)p * K + d + q];      // r^T A' lam
      const double lb = h[K + q] + s4[(size_t)p * K + q];          // (A lam)^T A' beta*
      grad.push_back(-2.0 * (rb + mu * (rl - lb)));
    }
  }
  *loss_out = loss;
  for (size_t k = 0; k < grad.size(); ++k) grad_out[k] = grad[k];
  CHECK_HIP(hipStreamSynchronize(st));
  return ok();
}

// ------------------------------------------------------------------ row-dependent coefficients
// Blocks sum_t a_t(x) L_t: each channel folded per feature into (S, C) as Eq. (2) folds a
// constant-coefficient operator, the per-row coefficients gathered into a T x P table.  The
// matrix is assembled to HBM (the Gram contracts the stored rows on the FP64 matrix cores;
// refinement products stream them), since a row-dependent coefficient on the cosine part does
// not fit the one-sine-per-entry form of the matrix-free passes.
struct VarSys {
  int d = 0, n = 0, n_blocks = 0, T = 0;
  int64_t P = 0;
  const double* W = nullptr;
  const double* b = nullptr;
  std::vector<int64_t> row0, rows;
  std::vector<double> weight;
  std::vector<int> n_ch;
  DevBuf X, row_block, S, C, acoef, rhs_w, terms, off, scale;
  VarGeo geo(double* A, double* At) const {
    VarGeo g;
    g.d = d;
    g.n = n;
    g.T = T;
    g.P = P;
    g.W = W;
    g.b = b;
    g.X = X.as<double>();
    g.row_block = row_block.as<int32_t>();
    g.S = S.as<double>();
    g.C = C.as<double>();
    g.acoef = acoef.as<double>();
    g.A = A;
    g.At = At;
    return g;
  }
  double* coef_row(int t, int64_t row) const { return acoef.as<double>() + (int64_t)t * P + row; }
};

Err check_vblocks(const flsq_vrows* blocks, int nb, int d, bool need_rhs, int max_ch) {
  if (nb < 1 || !blocks) return fail(FLSQ_EINVAL, "need at least one row block");
  if (nb > 64) return fail(FLSQ_EINVAL, "at most 64 row blocks");
  int64_t P = 0;
  for (int i = 0; i < nb; ++i) {
    const flsq_vrows& r = blocks[i];
    if (r.n_rows < 0) return fail(FLSQ_EINVAL, "block %d: n_rows < 0", i);
    if (r.n_rows > 0 && !r.x) return fail(FLSQ_EINVAL, "block %d: x is NULL", i);
    if (need_rhs && r.n_rows > 0 && !r.rhs) return fail(FLSQ_EINVAL, "block %d: rhs is NULL", i);
    if (!std::isfinite(r.weight)) return fail(FLSQ_ENONFINITE, "block %d: weight not finite", i);
    if (r.n_channels < 1 || r.n_channels > max_ch || !r.channels)
      return fail(FLSQ_EINVAL, "block %d: n_channels = %d outside [1, %d]", i, r.n_channels, max_ch);
    for (int t = 0; t < r.n_channels; ++t) CHECK_ERR(check_op(r.channels[t].op, d, i));
    P += r.n_rows;
  }
  if (P < 1) return fail(FLSQ_EINVAL, "no rows");
  if (P > (int64_t)0x7fffffff) return fail(FLSQ_EINVAL, "more than 2^31 - 1 rows");
  return ok();
}

Err build_var(flsq_ctx* c, VarSys& s, const flsq_basis* basis, const flsq_vrows* blocks, int nb, bool need_rhs,
              int max_ch = FLSQ_MAX_CHANNELS) {
  CHECK_ERR(check_basis(basis));
  CHECK_ERR(check_vblocks(blocks, nb, basis->d, need_rhs, max_ch));
  hipStream_t st = c->stream;
  s.d = basis->d;
  s.n = basis->n_feat;
  s.W = basis->W;
  s.b = basis->b;
  s.n_blocks = nb;
  s.row0.assign(nb, 0);
  s.rows.assign(nb, 0);
  s.weight.assign(nb, 0.0);
  s.n_ch.assign(nb, 0);
  s.T = 0;
  int64_t P = 0;
  for (int i = 0; i < nb; ++i) {
    s.row0[i] = P;
    s.rows[i] = blocks[i].n_rows;
    s.weight[i] = blocks[i].weight;
    s.n_ch[i] = blocks[i].n_channels;
    s.T = std::max(s.T, blocks[i].n_channels);
    P += blocks[i].n_rows;
  }
  s.P = P;
  const int d = s.d, n = s.n, T = s.T;
  const double norm = basis->normalize ? 1.0 / std::sqrt((double)n) : 1.0;
  CHECK_HIP(s.X.ensure(sizeof(double) * P * d));
  CHECK_HIP(s.row_block.ensure(sizeof(int32_t) * P));
  CHECK_HIP(s.acoef.ensure(sizeof(double) * T * P));
  CHECK_HIP(s.rhs_w.ensure(sizeof(double) * P));
  CHECK_HIP(s.S.ensure(sizeof(double) * nb * T * n));
  CHECK_HIP(s.C.ensure(sizeof(double) * nb * T * n));
  std::vector<VarTerm> tv;
  std::vector<int32_t> off(1, 0);
  std::vector<double> sc;
  for (int i = 0; i < nb; ++i) {
    const flsq_vrows& r = blocks[i];
    for (int t = 0; t < T; ++t) {
      if (t < r.n_channels) {
        const flsq_op& op = r.channels[t].op;
        for (int k = 0; k < op.n_terms; ++k) {
          VarTerm vt;
          memset(&vt, 0, sizeof vt);
          vt.coef = op.terms[k].coef;
          for (int q = 0; q < kMaxDim; ++q) vt.alpha[q] = op.terms[k].alpha[q];
          tv.push_back(vt);
        }
      }
      off.push_back((int32_t)tv.size());
      sc.push_back(r.weight * norm);
      if (r.n_rows == 0) continue;
      double* dst = s.coef_row(t, s.row0[i]);
      if (t < r.n_channels && r.channels[t].coef)
        CHECK_HIP(hipMemcpyAsync(dst, r.channels[t].coef, sizeof(double) * r.n_rows, hipMemcpyDeviceToDevice, st));
      else
        CHECK_HIP(launch_fill_f64(dst, r.n_rows, t < r.n_channels ? 1.0 : 0.0, st));
    }
    if (r.n_rows > 0) {
      CHECK_HIP(hipMemcpyAsync(s.X.as<double>() + s.row0[i] * d, r.x, sizeof(double) * d * r.n_rows,
                               hipMemcpyDeviceToDevice, st));
      CHECK_HIP(launch_fill_i32(s.row_block.as<int32_t>() + s.row0[i], r.n_rows, i, st));
      CHECK_HIP(launch_scale_copy(r.rhs, s.rhs_w.as<double>() + s.row0[i], r.n_rows, r.weight, st));  // NULL -> 0
    }
  }
  CHECK_HIP(s.terms.ensure(sizeof(VarTerm) * std::max<size_t>(1, tv.size())));
  CHECK_HIP(s.off.ensure(sizeof(int32_t) * off.size()));
  CHECK_HIP(s.scale.ensure(sizeof(double) * sc.size()));
  if (!tv.empty()) CHECK_ERR(stage_upload(c, s.terms.p, tv.data(), sizeof(VarTerm) * tv.size()));
  CHECK_ERR(stage_upload(c, s.off.p, off.data(), sizeof(int32_t) * off.size()));
  CHECK_ERR(stage_upload(c, s.scale.p, sc.data(), sizeof(double) * sc.size()));
  CHECK_HIP(launch_fold_var(s.W, n, d, s.terms.as<VarTerm>(), s.off.as<int32_t>(), s.scale.as<double>(), nb * T,
                            s.S.as<double>(), s.C.as<double>(), st));
  CHECK_ERR(check_finite_many(c, {FiniteItem{s.X.as<double>(), P * d, "collocation points"},
                                  FiniteItem{s.acoef.as<double>(), (int64_t)T * P, "channel coefficients"},
                                  FiniteItem{s.W, (int64_t)n * d, "W"}, FiniteItem{s.b, n, "b"},
                                  FiniteItem{need_rhs ? s.rhs_w.as<double>() : nullptr, P, "right-hand side"}}));
  return ok();
}

// G = At A (n x n, full) on the FP64 matrix cores, K = P split across workgroups.
Err stored_gram(flsq_ctx* c, const double* A, const double* At, int n, int64_t P, double* G) {
  GemmDesc h;
  memset(&h, 0, sizeof h);
  h.A = At;
  h.lda = (int)P;
  h.B = A;
  h.ldb = n;
  h.C = G;
  h.ldc = n;
  h.M = n;
  h.N = n;
  h.K = (int)P;
  h.tri = 0;
  GemmDesc* dd;
  CHECK_ERR(upload_descs(c, std::vector<GemmDesc>(1, h), &dd));
  double* work;
  const size_t we = (size_t)8 * n * n;
  CHECK_ERR(ws_get(c, "vg_work", we, &work));
  CHECK_HIP(hipEventRecord(c->ev0, c->stream));
  CHECK_HIP(launch_gemm_tri(dd, 1, n, n, (int)P, 1.0, work, we, c->stream));
  CHECK_HIP(hipEventRecord(c->ev1, c->stream));
  return ok();
}

// Tikhonov least squares with a stored matrix: Gram, Cholesky with shift retries, initial
// solve, CGLS refinement (one right-hand side Yw, P rows).
Err var_linear_solve(flsq_ctx* c, const double* A, const double* At, int n, int64_t P, const SolveParams& sp,
                     const double* Yw, double* beta, flsq_solve_info* info, bool* converged) {
  double *G, *U, *Xi, *cvec;
  CHECK_ERR(ws_get(c, "vG", (size_t)n * n, &G));
  CHECK_ERR(ws_get(c, "Ufac", (size_t)n * n, &U));
  CHECK_ERR(ws_get(c, "Xinv", (size_t)n * n, &Xi));
  CHECK_ERR(ws_get(c, "cvec", (size_t)n, &cvec));
  const double t0 = now_ms();
  CHECK_ERR(stored_gram(c, A, At, n, P, G));
  CHECK_HIP(hipStreamSynchronize(c->stream));
  const double t1 = now_ms();
  float kms = 0.f;
  CHECK_HIP(hipEventElapsedTime(&kms, c->ev0, c->ev1));
  c->last_gram_kernel_ms = kms;
  double shift = 0.0;
  int retries = 0;
  int boosted = 0, recalled = 0;
  CHECK_ERR(factor_with_retries(c, G, U, Xi, n, sp.mu, sp.shift_rel, &shift, &retries, sp.pivot_boost, &boosted,
                                &recalled));
  const double t2a = now_ms();
  bool second = false;
  if (want_second_pass(sp, retries + recalled + (boosted > 0 ? 1 : 0), nullptr, P, n)) {
    double shift2 = 0.0;
    int retries2 = 0;
    CHECK_ERR(second_pass_factor(c, A, P, n, sp.mu, Xi, &shift2, &retries2, &second));
    retries += retries2;
  }
  CHECK_HIP(hipStreamSynchronize(c->stream));
  const double t2 = now_ms();
  CHECK_HIP(launch_rowdot(At, n, P, P, Yw, nullptr, 1.0, 0.0, cvec, c->stream));
  CHECK_ERR(chol_solve(c, Xi, n, cvec, beta, 1));
  RefineOut ro;
  const bool lazy = sp.second_pass == 0 && !second && second_pass_allowed(sp, nullptr, P, n) &&
                    2.0 * (double)P * n * n <= kLazySecondPassFlops;
  double t_second = 0.0;
  auto make_A = [&](const double** Aout) -> Err {
    *Aout = A;
    return ok();
  };
  bool late = false;
  CHECK_ERR(refine_lazy(c, DenseOp(A, At, n, P), sp, lazy, make_A, Xi, Yw, 1, beta, info != nullptr,
                        info != nullptr && sp.report_grad, &ro, &late, &t_second));
  CHECK_HIP(hipStreamSynchronize(c->stream));
  if (late) second = true;
  if (info) {
    info->t_gram_ms = t1 - t0;
    info->t_chol_ms = t2 - t1;
    info->shift = shift;
    info->chol_retries = retries;
    info->boosted_pivots = boosted;
    info->shift_recalled = recalled;
    info->t_gram_kernel_ms = c->last_gram_kernel_ms;
    info->refine_iters = ro.iters;
    info->grad_norm0 = ro.grad0;
    info->grad_norm = ro.grad;
    info->last_step_rel = ro.last_step;
    info->t_refine_ms = now_ms() - t2;
    info->second_pass = second ? 1 : 0;
    info->t_second_pass_ms = late ? t_second : (second ? t2 - t2a : 0.0);
  }
  if (converged) *converged = ro.converged;
  return ok();
}

Err assemble_var_dev(flsq_ctx* c, const VarSys& s, const char* nameA, const char* nameAt, double** A, double** At) {
  CHECK_ERR(ws_get(c, nameA, (size_t)s.P * s.n, A));
  *At = nullptr;
  if (nameAt) CHECK_ERR(ws_get(c, nameAt, (size_t)s.P * s.n, At));
  CHECK_HIP(launch_assemble_var(s.geo(*A, *At), c->stream));
  return ok();
}

Err linear_var_impl(flsq_ctx* c, const flsq_basis* basis, const flsq_vrows* blocks, int nb, const flsq_solve_opts* o,
                    double* beta, flsq_solve_info* info, bool* converged) {
  if (!beta) return fail(FLSQ_EINVAL, "beta_out is NULL");
  SolveParams sp = params_of(o);
  CHECK_ERR(check_params(sp));
  if (sp.prec != FLSQ_PREC_FP64) return fail(FLSQ_EINVAL, "row-dependent coefficients: only FLSQ_PREC_FP64");
  if (info) memset(info, 0, sizeof *info);
  const double t0 = now_ms();
  VarSys s;
  CHECK_ERR(build_var(c, s, basis, blocks, nb, true));
  double *A, *At;
  CHECK_ERR(assemble_var_dev(c, s, "vA", "vAt", &A, &At));
  CHECK_ERR(var_linear_solve(c, A, At, s.n, s.P, sp, s.rhs_w.as<double>(), beta, info, converged));
  if (info) info->t_total_ms = now_ms() - t0;
  return check_finite_dev(c, beta, s.n, "beta");
}

Err newton_var_impl(flsq_ctx* c, const flsq_basis* basis, const flsq_vrows* blocks, int nb, int nl_block,
                    const flsq_nonlin_grad* nl, const flsq_newton_opts* o, double tol_du, double* beta,
                    flsq_newton_trace* tr, bool* converged) {
  if (!o) return fail(FLSQ_EINVAL, "opts is NULL");
  if (!beta) return fail(FLSQ_EINVAL, "beta_inout is NULL");
  if (o->max_iter < 0 || o->max_iter > 64) return fail(FLSQ_EINVAL, "max_iter outside [0, 64]");
  if (o->max_halvings < 0 || o->max_halvings > 60) return fail(FLSQ_EINVAL, "max_halvings outside [0, 60]");
  if (!(o->armijo_c >= 0.0 && o->armijo_c < 1.0)) return fail(FLSQ_EINVAL, "armijo_c outside [0, 1)");
  if (!(tol_du >= 0.0)) return fail(FLSQ_EINVAL, "tol_du must be >= 0");
  SolveParams sp = params_of(&o->lin);
  CHECK_ERR(check_params(sp));
  if (sp.prec != FLSQ_PREC_FP64) return fail(FLSQ_EINVAL, "row-dependent coefficients: only FLSQ_PREC_FP64");
  CHECK_ERR(check_basis(basis));
  const int d = basis->d;
  if (!nl) return fail(FLSQ_EINVAL, "nonlinearity is NULL");
  if (nl->n_poly < 0 || nl->n_poly > kMaxNlTerms || (nl->n_poly > 0 && !nl->poly))
    return fail(FLSQ_EINVAL, "nonlinearity: n_poly in [0, %d]", kMaxNlTerms);
  if (nl->n_adv < 0 || nl->n_adv > kMaxNlTerms || (nl->n_adv > 0 && (!nl->adv_coef || !nl->adv_pow || !nl->adv_axis)))
    return fail(FLSQ_EINVAL, "nonlinearity: n_adv in [0, %d] with its arrays", kMaxNlTerms);
  if (!std::isfinite(nl->exp_coef)) return fail(FLSQ_ENONFINITE, "exponential coefficient not finite");
  if (nl->n_poly + nl->n_adv < 1 && nl->exp_coef == 0.0) return fail(FLSQ_EINVAL, "nonlinearity has no terms");
  NlSpec spec;
  memset(&spec, 0, sizeof spec);
  spec.exp_coef = nl->exp_coef;
  spec.n_poly = nl->n_poly;
  for (int k = 0; k < nl->n_poly; ++k) {
    if (!std::isfinite(nl->poly[k])) return fail(FLSQ_ENONFINITE, "nonlinearity coefficient not finite");
    spec.poly[k] = nl->poly[k];
  }
  std::vector<int> axes;
  spec.n_adv = nl->n_adv;
  for (int t = 0; t < nl->n_adv; ++t) {
    if (!std::isfinite(nl->adv_coef[t])) return fail(FLSQ_ENONFINITE, "advection coefficient not finite");
    if (nl->adv_pow[t] < 0 || nl->adv_pow[t] > 16) return fail(FLSQ_EINVAL, "advection power outside [0, 16]");
    if (nl->adv_axis[t] < 0 || nl->adv_axis[t] >= d) return fail(FLSQ_EINVAL, "advection axis outside [0, d)");
    int sl = (int)(std::find(axes.begin(), axes.end(), nl->adv_axis[t]) - axes.begin());
    if (sl == (int)axes.size()) axes.push_back(nl->adv_axis[t]);
    spec.c[t] = nl->adv_coef[t];
    spec.m[t] = nl->adv_pow[t];
    spec.slot[t] = sl;
  }
  const int ns = (int)axes.size();
  spec.n_slots = ns;
  if (nl_block < 0 || nl_block >= nb || !blocks)
    return fail(FLSQ_EINVAL, "nonlin_block %d outside [0, %d)", nl_block, nb);
  // linear operator A_L (and its transpose for the warm start)
  VarSys L;
  CHECK_ERR(build_var(c, L, basis, blocks, nb, true));
  const int n = L.n;
  const int64_t P = L.P;
  const int64_t nl0 = L.row0[nl_block], nln = L.rows[nl_block];
  const double w_nl = L.weight[nl_block];
  hipStream_t st = c->stream;
  double *AL, *ALt;
  CHECK_ERR(assemble_var_dev(c, L, "nv_AL", "nv_ALt", &AL, &ALt));
  // evaluation rows E: u at every row (identity, weight 1), then d_axis u on the nonlinear rows
  flsq_term id_term;
  memset(&id_term, 0, sizeof id_term);
  id_term.coef = 1.0;
  std::vector<flsq_term> dterms(ns, id_term);
  for (int s2 = 0; s2 < ns; ++s2) dterms[s2].alpha[axes[s2]] = 1;
  std::vector<flsq_channel> ech(1 + ns);
  ech[0].op.terms = &id_term;
  ech[0].op.n_terms = 1;
  ech[0].coef = nullptr;
  for (int s2 = 0; s2 < ns; ++s2) {
    ech[1 + s2].op.terms = &dterms[s2];
    ech[1 + s2].op.n_terms = 1;
    ech[1 + s2].coef = nullptr;
  }
  std::vector<flsq_vrows> eb;
  for (int i = 0; i < nb; ++i) {
    flsq_vrows r = blocks[i];
    r.weight = 1.0;
    r.rhs = nullptr;
    r.n_channels = 1;
    r.channels = &ech[0];
    eb.push_back(r);
  }
  for (int s2 = 0; s2 < ns; ++s2) {
    flsq_vrows r = blocks[nl_block];
    r.weight = 1.0;
    r.rhs = nullptr;
    r.n_channels = 1;
    r.channels = &ech[1 + s2];
    eb.push_back(r);
  }
  VarSys E;
  CHECK_ERR(build_var(c, E, basis, eb.data(), (int)eb.size(), false));
  const int64_t PE = E.P;
  double *EA, *dummy;
  CHECK_ERR(assemble_var_dev(c, E, "nv_E", nullptr, &EA, &dummy));
  // Jacobian system: the nonlinear block gains (identity, dN/du) and (d_axis, dN/d(d_axis u))
  std::vector<flsq_channel> jch(blocks[nl_block].channels, blocks[nl_block].channels + blocks[nl_block].n_channels);
  const int t_rho = (int)jch.size();
  jch.push_back(ech[0]);
  for (int s2 = 0; s2 < ns; ++s2) jch.push_back(ech[1 + s2]);
  std::vector<flsq_vrows> jb(blocks, blocks + nb);
  jb[nl_block].channels = jch.data();
  jb[nl_block].n_channels = (int32_t)jch.size();
  VarSys Jsys;
  CHECK_ERR(build_var(c, Jsys, basis, jb.data(), nb, true, FLSQ_MAX_CHANNELS + 1 + kMaxNlTerms));
  double* rho_dst = Jsys.coef_row(t_rho, nl0);
  double* kap_dst = Jsys.coef_row(t_rho + 1, nl0);
  double *R, *Rt, *UE, *UEt, *negR, *delta, *bt, *tmp, *dots, *dwork;
  CHECK_ERR(ws_get(c, "nv_R", (size_t)P, &R));
  CHECK_ERR(ws_get(c, "nv_Rt", (size_t)P, &Rt));
  CHECK_ERR(ws_get(c, "nv_UE", (size_t)PE, &UE));
  CHECK_ERR(ws_get(c, "nv_UEt", (size_t)PE, &UEt));
  CHECK_ERR(ws_get(c, "nv_negR", (size_t)P, &negR));
  CHECK_ERR(ws_get(c, "nv_delta", (size_t)n, &delta));
  CHECK_ERR(ws_get(c, "nv_bt", (size_t)n, &bt));
  CHECK_ERR(ws_get(c, "nv_tmp", (size_t)P, &tmp));
  CHECK_ERR(ws_get(c, "nv_dots", 8, &dots));
  CHECK_ERR(ws_get(c, "nv_dwork", 1024, &dwork));
  const double* data_w = L.rhs_w.as<double>();
  auto dot1 = [&](const double* x, const double* y, int64_t len, double* out) -> Err {
    CHECK_HIP(launch_dot_cols(x, y, len, 1, dots, dwork, st));
    CHECK_ERR(read_back(c, out, dots, sizeof(double)));
    return ok();
  };
  // R = A_L b - data + w N(u, grad u) on the nonlinear rows; the Jacobian coefficients of the
  // point b go to the Jacobian system's coefficient table
  auto residual = [&](const double* b, double* Rout, double* Uout, double* nrm) -> Err {
    CHECK_HIP(launch_rowdot(EA, PE, n, n, b, nullptr, 1.0, 0.0, Uout, st));
    CHECK_HIP(launch_rowdot(AL, P, n, n, b, data_w, 1.0, -1.0, Rout, st));
    CHECK_HIP(launch_nl_var(spec, Uout, P, nl0, nln, w_nl, Rout, rho_dst, ns ? kap_dst : nullptr, P, st));
    double h = 0.0;
    CHECK_ERR(dot1(Rout, Rout, P, &h));
    *nrm = std::sqrt(h);
    if (!std::isfinite(*nrm)) return fail(FLSQ_ENONFINITE, "Newton residual is not finite");
    return ok();
  };
  const double t0 = now_ms();
  SolveParams spk = sp;
  flsq_solve_info sinfo;
  if (o->warm_start) {
    CHECK_ERR(var_linear_solve(c, AL, ALt, n, P, spk, data_w, beta, &sinfo, nullptr));
    spk.shift_rel = std::max(spk.shift_rel, sinfo.shift);
  }
  if (tr) memset(tr, 0, sizeof *tr);
  *converged = false;
  double nR = 0.0;
  CHECK_ERR(residual(beta, R, UE, &nR));
  std::vector<double> one(1, 1.0);
  double *J, *Jt;
  // Newton steps need no fully refined step (the outer iteration corrects it): the automatic
  // second pass is left to the warm start; an explicit request still applies to every step.
  if (spk.second_pass == 0) spk.second_pass = -1;
  for (int it = 0; it < o->max_iter; ++it) {
    CHECK_ERR(assemble_var_dev(c, Jsys, "nv_J", "nv_Jt", &J, &Jt));
    CHECK_HIP(launch_scale_copy(R, negR, P, -1.0, st));
    const double ts = now_ms();
    CHECK_ERR(var_linear_solve(c, J, Jt, n, P, spk, negR, delta, &sinfo, nullptr));
    const double t_solve = now_ms() - ts;
    spk.shift_rel = std::max(spk.shift_rel, sinfo.shift);
    double alpha = 1.0, nRt = 0.0;
    int halv = 0;
    for (;;) {
      CHECK_HIP(hipMemcpyAsync(bt, beta, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
      one[0] = alpha;
      CHECK_HIP(launch_axpy_cols(cols(one), delta, bt, n, 1, 1.0, st));
      CHECK_ERR(residual(bt, Rt, UEt, &nRt));
      if (nRt <= (1.0 - o->armijo_c * alpha) * nR || halv >= o->max_halvings) break;
      alpha *= 0.5;
      ++halv;
    }
    double dd = 0.0, du2 = 0.0, un2 = 0.0;
    CHECK_ERR(dot1(delta, delta, n, &dd));
    const double step = alpha * std::sqrt(dd);
    // ||Delta u|| / ||u|| over every collocation row
    CHECK_HIP(hipMemcpyAsync(tmp, UEt, sizeof(double) * P, hipMemcpyDeviceToDevice, st));
    one[0] = 1.0;
    CHECK_HIP(launch_axpy_cols(cols(one), UE, tmp, P, 1, -1.0, st));
    CHECK_ERR(dot1(tmp, tmp, P, &du2));
    CHECK_ERR(dot1(UEt, UEt, P, &un2));
    const double du_rel = std::sqrt(du2) / std::max(std::sqrt(un2), 1e-300);
    if (tr) {
      tr->res_norm[it] = nR;
      tr->alpha[it] = alpha;
      tr->halvings[it] = halv;
      tr->step_norm[it] = step;
      tr->du_rel[it] = du_rel;
      tr->refine_iters[it] = sinfo.refine_iters;
      tr->shift[it] = sinfo.shift;
      tr->t_solve_ms[it] = t_solve;
      tr->factored[it] = 1;
      tr->iters = it + 1;
    }
    CHECK_HIP(hipMemcpyAsync(beta, bt, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    std::swap(R, Rt);
    std::swap(UE, UEt);
    nR = nRt;
    if (du_rel < tol_du || step < o->tol_dbeta) {
      *converged = true;
      break;
    }
  }
  CHECK_HIP(hipStreamSynchronize(st));
  if (tr) {
    tr->converged = *converged ? 1 : 0;
    tr->t_total_ms = now_ms() - t0;
  }
  return check_finite_dev(c, beta, n, "beta");
}

}  // namespace

extern "C" {

flsq_status flsq_solve_newton(flsq_ctx* ctx, const flsq_basis* basis, const flsq_rows* blocks, int32_t n_blocks,
                              int32_t nonlin_block, const flsq_nonlin* nonlin, const flsq_newton_opts* opts,
                              double* beta_inout, flsq_newton_trace* trace) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  bool conv = false;
  Err e = newton_impl(ctx, basis, blocks, n_blocks, nonlin_block, nonlin, opts, beta_inout, trace, &conv);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (!conv && opts->tol_dbeta > 0.0)
    return finish(ctx, fail(FLSQ_ENOCONV, "Newton: ||alpha delta|| did not fall below tol_dbeta in %d steps",
                            opts->max_iter));
  return finish(ctx, ok());
}

flsq_status flsq_inverse_prepare(flsq_ctx* ctx, flsq_factor* F, int64_t n_src_rows, int64_t n_obs,
                                 const double* x_obs) {
  if (!ctx || !F) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  return finish(ctx, inverse_prepare_impl(ctx, F, n_src_rows, n_obs, x_obs));
}

flsq_status flsq_inverse_loss_grad(flsq_ctx* ctx, const flsq_factor* F, int64_t n_src_rows, double src_weight,
                                   int32_t n_lap_dims, const double* thetas, int32_t K, int64_t n_obs,
                                   const double* x_obs, const double* data, double* loss_out,
                                   double* grad_theta_out, double* grad_kappa_out) {
  if (!ctx || !F) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  Err e = inverse_impl(ctx, const_cast<flsq_factor*>(F), n_src_rows, src_weight, n_lap_dims, thetas, K, n_obs, x_obs,
                       data, loss_out, grad_theta_out, grad_kappa_out);
  return finish(ctx, e);
}

flsq_status flsq_bandwidth_loss_grad(flsq_ctx* ctx, const flsq_basis* base, const double* L, const flsq_rows* blocks,
                                     int32_t n_blocks, const flsq_solve_opts* opts, double* beta_out, double* loss_out,
                                     double* grad_out) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  Err e = bandwidth_impl(ctx, base, L, blocks, n_blocks, opts, beta_out, loss_out, grad_out);
  return finish(ctx, e);
}

flsq_status flsq_assemble_var(flsq_ctx* ctx, const flsq_basis* basis, const flsq_vrows* blocks, int32_t n_blocks,
                              double* A_out, double* rhs_out) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!A_out) return finish(ctx, fail(FLSQ_EINVAL, "A_out is NULL"));
  VarSys s;
  Err e = build_var(ctx, s, basis, blocks, n_blocks, rhs_out != nullptr);
  if (e.st == FLSQ_OK) {
    hipError_t he = launch_assemble_var(s.geo(A_out, nullptr), ctx->stream);
    if (he == hipSuccess && rhs_out)
      he = hipMemcpyAsync(rhs_out, s.rhs_w.p, sizeof(double) * s.P, hipMemcpyDeviceToDevice, ctx->stream);
    if (he == hipSuccess) he = hipStreamSynchronize(ctx->stream);
    if (he != hipSuccess) e = fail(FLSQ_EHIP, "assemble_var: %s", hipGetErrorString(he));
  }
  return finish(ctx, e);
}

flsq_status flsq_solve_linear_var(flsq_ctx* ctx, const flsq_basis* basis, const flsq_vrows* blocks,
                                  int32_t n_blocks, const flsq_solve_opts* opts, double* beta_out,
                                  flsq_solve_info* info) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  bool conv = true;
  Err e = linear_var_impl(ctx, basis, blocks, n_blocks, opts, beta_out, info, &conv);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (!conv && opts->refine_tol > 0.0)
    return finish(ctx, fail(FLSQ_ENOCONV, "refinement did not reach refine_tol in %d iterations", opts->max_refine));
  return finish(ctx, ok());
}

flsq_status flsq_solve_newton_var(flsq_ctx* ctx, const flsq_basis* basis, const flsq_vrows* blocks,
                                  int32_t n_blocks, int32_t nonlin_block, const flsq_nonlin_grad* nonlin,
                                  const flsq_newton_opts* opts, double tol_du, double* beta_inout,
                                  flsq_newton_trace* trace) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  bool conv = false;
  Err e = newton_var_impl(ctx, basis, blocks, n_blocks, nonlin_block, nonlin, opts, tol_du, beta_inout, trace, &conv);
  if (e.st != FLSQ_OK) return finish(ctx, e);
  if (!conv && (tol_du > 0.0 || opts->tol_dbeta > 0.0))
    return finish(ctx, fail(FLSQ_ENOCONV, "Newton: neither stopping rule met in %d steps", opts->max_iter));
  return finish(ctx, ok());
}

flsq_status flsq_adam_step(flsq_ctx* ctx, double* params, const double* grads, double* m, double* v, int32_t K,
                           int32_t P, int32_t t, double lr, double b1, double b2, double eps, int32_t clamp_col,
                           double clamp_min, double weight_decay) {
  if (!ctx) return FLSQ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "hipSetDevice failed"));
  if (!params || !grads || !m || !v) return finish(ctx, fail(FLSQ_EINVAL, "NULL argument"));
  if (K < 1 || P < 1 || t < 1) return finish(ctx, fail(FLSQ_EINVAL, "K, P and t must be >= 1"));
  if (clamp_col >= P) return finish(ctx, fail(FLSQ_EINVAL, "clamp_col >= P"));
  if (!std::isfinite(weight_decay) || weight_decay < 0.0) return finish(ctx, fail(FLSQ_EINVAL, "weight_decay < 0"));
  hipError_t he = launch_adam(params, grads, m, v, K, P, t, lr, b1, b2, eps, clamp_col, clamp_min, weight_decay,
                              ctx->stream);
  if (he != hipSuccess) return finish(ctx, fail(FLSQ_EHIP, "adam: %s", hipGetErrorString(he)));
  return finish(ctx, ok());
}

}  // extern "C"
