// libdls: the C ABI declared in include/dls.h.
//
// Compression is split in a device half (dls_encode: plan upload, Gram,
// eigensolve + rank, offset scan, projection / quantization / residual codes)
// and a host half (dls_finalize: copy the packed payload to host, sort the
// escapes, deflate each batch of 1000 blocks on host threads, write the
// header and batch table, Sec. 2.7.2).  Decompression (Alg. 2) inflates on
// host threads and rebuilds the field on the device.
#include <hip/hip_runtime.h>
#include <zlib.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "../../include/dls.h"
#include "dls_internal.h"
#include "dls_kernels.h"

using namespace dls;

namespace {

thread_local std::string g_err;

dls_status fail(dls_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(e_ == hipErrorOutOfMemory ? DLS_ENOMEM : DLS_EDEVICE,            \
                  std::string(#expr) + ": " + hipGetErrorString(e_));              \
  } while (0)

// Device (re)allocations by DevBuf, process-wide: a captured launch sequence
// stays valid only while every buffer it names stays where it was.
std::atomic<uint64_t> g_alloc_epoch{0};
// words of the key of a captured device-driven encode sequence
constexpr int kDdKey = 16;

struct DevBuf {
  void* p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) {
      (void)hipFree(p);
      ++g_alloc_epoch;
    }
    p = nullptr;
    n = 0;
  }
  hipError_t ensure(size_t bytes) {
    if (bytes == 0) bytes = 16;
    if (bytes <= n) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, bytes);
    if (e == hipSuccess) n = bytes;
    else p = nullptr;
    ++g_alloc_epoch;
    return e;
  }
  // at least `bytes`, contents not kept
  hipError_t grow(size_t bytes) { return ensure(bytes); }
  template <typename T>
  T* as() const { return static_cast<T*>(p); }
};

int worker_count() {
  unsigned n = std::thread::hardware_concurrency();
  if (const char* s = std::getenv("DLS_HOST_THREADS")) n = unsigned(std::max(1, atoi(s)));
  return int(std::max(1u, std::min(n, 64u)));
}

template <typename F>
void parallel_for(int64_t n, F&& fn) {
  const int nw = int(std::min<int64_t>(worker_count(), std::max<int64_t>(n, 1)));
  std::atomic<int64_t> next{0};
  auto body = [&]() {
    for (int64_t i = next++; i < n; i = next++) fn(i);
  };
  std::vector<std::thread> th;
  for (int w = 1; w < nw; ++w) th.emplace_back(body);
  body();
  for (auto& t : th) t.join();
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

dls_status validate(const dls_params* in, Problem& p) {
  if (in == nullptr) return fail(DLS_EINVAL, "params is NULL");
  if (in->struct_size != sizeof(dls_params)) return fail(DLS_EINVAL, "params.struct_size mismatch");
  p.nvars = in->nvars;
  p.nx = in->nx; p.ny = in->ny; p.nz = in->nz; p.nt = in->nt;
  p.dtype = in->dtype;
  p.px = in->px; p.py = in->py; p.pz = in->pz; p.pmin = in->pmin;
  p.window = in->window;
  p.precision = in->precision;
  p.flags = in->flags;
  if (p.nvars < 1 || p.nvars > 65536) return fail(DLS_EINVAL, "nvars out of range");
  const int64_t lim = int64_t(1) << 31;
  if (p.nx < 1 || p.ny < 1 || p.nz < 1 || p.nt < 1 || p.nx >= lim || p.ny >= lim || p.nz >= lim || p.nt >= lim)
    return fail(DLS_EINVAL, "grid sizes must be in [1, 2^31)");
  if (p.dtype != DLS_F32 && p.dtype != DLS_F64) return fail(DLS_EINVAL, "dtype must be DLS_F32 or DLS_F64");
  if (p.window < 1 || p.window > 32) return fail(DLS_EINVAL, "window must be in [1, 32]");
  if (p.px < 1 || p.px > 32 || p.py < 1 || p.py > 32 || p.pz < 1 || p.pz > 32)
    return fail(DLS_EINVAL, "patch edges must be in [1, 32]");
  if (p.nz == 1 && p.pz != 1) return fail(DLS_EINVAL, "pz must be 1 for a 2D field");
  if (in->r_max < 0 || in->r_max > 32) return fail(DLS_EINVAL, "r_max must be in [0, 32]");
  p.r_max = in->r_max > 0 ? in->r_max : std::min(p.window, 32);
  if (p.flags & ~uint32_t(DLS_ADAPTIVE | DLS_LEARNED | DLS_PERSISTENT | DLS_L2 | DLS_GLOBAL))
    return fail(DLS_EINVAL, "unknown flags");
  if ((p.flags & DLS_L2) && (p.flags & DLS_LEARNED)) return fail(DLS_EINVAL, "DLS_L2 does not take DLS_LEARNED");
  if (p.flags & DLS_GLOBAL) {
    if (p.flags & (DLS_ADAPTIVE | DLS_LEARNED | DLS_L2))
      return fail(DLS_EINVAL, "DLS_GLOBAL does not take DLS_ADAPTIVE, DLS_LEARNED or DLS_L2");
    if (p.window != 1) return fail(DLS_EINVAL, "DLS_GLOBAL encodes every snapshot on its own: window must be 1");
    if (int64_t(p.px) * p.py * p.pz > kGbMaxM) return fail(DLS_EINVAL, "DLS_GLOBAL needs px * py * pz <= 1024");
    if (p.px > p.nx || p.py > p.ny || p.pz > p.nz) return fail(DLS_EINVAL, "DLS_GLOBAL needs the patch inside the grid");
    if (in->basis < DLS_BASIS_SVD || in->basis > DLS_BASIS_RANDOM) return fail(DLS_EINVAL, "unknown basis kind");
    p.basis = in->basis;
    p.seed = in->seed;
  }
  if (in->warm_iters < 0 || in->warm_iters > 8) return fail(DLS_EINVAL, "warm_iters must be in [0, 8]");
  if (in->rank_margin < 0 || in->rank_margin > 8) return fail(DLS_EINVAL, "rank_margin must be in [0, 8]");
  if ((p.flags & DLS_LEARNED) && p.window > 16) return fail(DLS_EINVAL, "DLS_LEARNED needs window <= 16");
  if (p.precision != DLS_PREC_FP32 && p.precision != DLS_PREC_BF16)
    return fail(DLS_EINVAL, "unknown precision");
  if (p.flags & DLS_ADAPTIVE) {
    if (!is_pow2(p.px) || p.py != p.px || p.pz != (p.nz > 1 ? p.px : 1))
      return fail(DLS_EINVAL, "adaptive plan needs px = py (= pz in 3D), a power of two");
    if (!is_pow2(p.pmin) || p.pmin > p.px) return fail(DLS_EINVAL, "pmin must be a power of two <= px");
  }
  if (in->abs_eps == nullptr) return fail(DLS_EINVAL, "abs_eps is NULL");
  p.eps.assign(in->abs_eps, in->abs_eps + p.nvars);
  for (double e : p.eps)
    if (!(e > 0.0) || !std::isfinite(e)) return fail(DLS_EINVAL, "abs_eps must be finite and > 0");
  return DLS_OK;
}

VarConst var_const(double eps) {
  VarConst k;
  k.eps = eps;
  k.c = std::ldexp(eps, -kBasisBits);
  k.inv_eps = 1.0 / eps;
  k.inv2eps = 1.0 / (2.0 * eps);
  k.inv_eps_f = float(k.inv_eps);
  k.pad = 0.f;
  return k;
}

int slice_points(const Problem& p) {
  return (p.dtype == DLS_F32 && p.wpad() == 16) ? 1024 : 512;
}

bool same_layout(const Problem& a, const Problem& b) {
  return a.nvars == b.nvars && a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.nt == b.nt &&
         a.dtype == b.dtype && a.px == b.px && a.py == b.py && a.pz == b.pz &&
         a.window == b.window && a.flags == b.flags && a.pmin == b.pmin;
}

}  // namespace

struct dls_model {
  int device = 0;
  DevBuf params, norm, m, v, grad;
  DevBuf packed;           // bf16 weights in the fused forward's LDS layout
  bool packed_valid = false;
  uint64_t version = 0;    // bumped whenever the parameters change
  int64_t step = 0;
  DevBuf z, h1, h2, out, gout, dh2, dh1, loss;  // workspace for a batch
  int64_t ws_n = 0;
};

namespace {
static_assert(kNParam == DLS_MODEL_NPARAM, "parameter count");

// inference forward (fused kernel); packs the bf16 weights after a change
dls_status model_infer(dls_model* m, const float* feat, int64_t n, float* out, hipStream_t s) {
  if (!m->packed_valid) {
    HIP_TRY(m->packed.ensure(kPackedWeightBytes));
    HIP_TRY(launch_pack_weights(m->params.as<float>(), m->packed.as<short>(), s));
    m->packed_valid = true;
  }
  HIP_TRY(launch_mlp_forward(feat, n, m->norm.as<float>(), m->params.as<float>(), m->packed.as<short>(), out, s));
  return DLS_OK;
}

dls_status model_workspace(dls_model* m, int64_t n) {
  if (n <= m->ws_n) return DLS_OK;
  HIP_TRY(m->z.ensure(size_t(n) * kNF * 4));
  HIP_TRY(m->h1.ensure(size_t(n) * kH * 4));
  HIP_TRY(m->h2.ensure(size_t(n) * kH * 4));
  HIP_TRY(m->out.ensure(size_t(n) * kNO * 4));
  HIP_TRY(m->gout.ensure(size_t(n) * kNO * 4));
  HIP_TRY(m->dh2.ensure(size_t(n) * kH * 4));
  HIP_TRY(m->dh1.ensure(size_t(n) * kH * 4));
  HIP_TRY(m->loss.ensure(size_t(n) * 4));
  m->ws_n = n;
  return DLS_OK;
}

// forward pass into m->z, h1, h2, and `out` (n x 272)
dls_status model_forward(dls_model* m, const float* feat, int64_t n, bool bf16, float* out, hipStream_t s) {
  const float* P = m->params.as<float>();
  HIP_TRY(launch_normalize(feat, n, m->norm.as<float>(), m->z.as<float>(), s));
  HIP_TRY(launch_gemm(false, false, bf16, m->z.as<float>(), kNF, P + kOffW1, kH, m->h1.as<float>(), kH, int(n), kH,
                      kNF, P + kOffb1, 1, s));
  HIP_TRY(launch_gemm(false, false, bf16, m->h1.as<float>(), kH, P + kOffW2, kH, m->h2.as<float>(), kH, int(n), kH,
                      kH, P + kOffb2, 1, s));
  HIP_TRY(launch_gemm(false, false, bf16, m->h2.as<float>(), kH, P + kOffW3, kNO, out, kNO, int(n), kNO, kH,
                      P + kOffb3, 0, s));
  return DLS_OK;
}

// forward + loss + backward into m->grad; *loss_out = batch mean loss
dls_status model_backprop(dls_model* m, const float* feat, const int32_t* rank, const float* basis, const int32_t* wb,
                          int64_t n, bool bf16, float* loss_out, hipStream_t s) {
  if (dls_status st = model_workspace(m, n)) return st;
  if (dls_status st = model_forward(m, feat, n, bf16, m->out.as<float>(), s)) return st;
  const float* P = m->params.as<float>();
  float* G = m->grad.as<float>();
  HIP_TRY(launch_loss(m->out.as<float>(), rank, basis, wb, n, m->gout.as<float>(), m->loss.as<float>(), s));
  // dW3 = h2^T gout, db3 = colsum(gout), dh2 = gout W3^T * relu'(h2)
  HIP_TRY(launch_gemm(true, false, bf16, m->h2.as<float>(), kH, m->gout.as<float>(), kNO, G + kOffW3, kNO, kH, kNO,
                      int(n), nullptr, 0, s));
  HIP_TRY(launch_colsum(m->gout.as<float>(), n, kNO, G + kOffb3, s));
  HIP_TRY(launch_gemm(false, true, bf16, m->gout.as<float>(), kNO, P + kOffW3, kNO, m->dh2.as<float>(), kH, int(n), kH,
                      kNO, nullptr, 0, s));
  HIP_TRY(launch_relu_mask(m->dh2.as<float>(), m->h2.as<float>(), n * kH, s));
  HIP_TRY(launch_gemm(true, false, bf16, m->h1.as<float>(), kH, m->dh2.as<float>(), kH, G + kOffW2, kH, kH, kH, int(n),
                      nullptr, 0, s));
  HIP_TRY(launch_colsum(m->dh2.as<float>(), n, kH, G + kOffb2, s));
  HIP_TRY(launch_gemm(false, true, bf16, m->dh2.as<float>(), kH, P + kOffW2, kH, m->dh1.as<float>(), kH, int(n), kH,
                      kH, nullptr, 0, s));
  HIP_TRY(launch_relu_mask(m->dh1.as<float>(), m->h1.as<float>(), n * kH, s));
  HIP_TRY(launch_gemm(true, false, bf16, m->z.as<float>(), kNF, m->dh1.as<float>(), kH, G + kOffW1, kH, kNF, kH, int(n),
                      nullptr, 0, s));
  HIP_TRY(launch_colsum(m->dh1.as<float>(), n, kH, G + kOffb1, s));
  if (loss_out != nullptr) {
    std::vector<float> l(n);
    HIP_TRY(hipMemcpyAsync(l.data(), m->loss.p, size_t(n) * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    double sum = 0.0;
    for (float v : l) sum += v;
    *loss_out = float(sum / double(n));
  }
  return DLS_OK;
}
}  // namespace

struct dls_ctx {
  int device = 0;
  Problem prob;
  bool plan_valid = false;
  Plan plan;
  int64_t plan_warm_blocks = 0;  // blocks small enough for the warm start
  int64_t plan_min_points = 0;   // smallest block of the plan (points)
  int64_t plan_qv_r1 = 0, plan_qa_r1 = 0;  // payload bytes if every block had rank 1
  bool r1_valid = false;         // r1_off holds the plan's static rank-1 payload offsets
  DevBuf r1_off;                 // [nblocks] qV then [nblocks] qA offsets of the rank-1 payload
  DevBuf fused;                  // fused-encode state: arrivals, verdicts, deferred list, counters
  unsigned long long* hfused = nullptr;  // pinned host copy of the fused counters
  int64_t nfast_accept = 0, ndeferred = 0;
  int64_t nesc_slots = 0;        // escape list entries to read (dropped ones included)
  int launch_mode = 0;           // 0 host-driven, 1 device-driven, 2 fused single pass
  bool fused_declined = false;   // the sketch predicted too many deferred blocks
  int64_t npredicted = 0, npruned = 0;
  bool split_valid = false;       // large / small slice lists of the plan
  int64_t split_nlarge = 0, split_nsmall = 0;
  DevBuf split_lists;
  bool feat_valid = false;        // the plan's block lists of the feature kernels
  int64_t feat_n[3] = {0, 0, 0};
  DevBuf feat_lists;
  DevBuf desc, items, item_start, code_off, gram, rank, lam, basis;
  DevBuf qv_size, qa_size, qv_off, qa_off, scan_tmp, qv, qa, codes, coef;
  DevBuf esc_key, esc_val, counters, vconst, eps_v, cls_lists, reject_list;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipEvent_t evs[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};  // gram, eigen, scan ends; encode start; plan start
  double stage_ms[5] = {0, 0, 0, 0, 0};
  // around the fused kernel and around the Jacobi launch of the last encode
  hipEvent_t evf[2] = {nullptr, nullptr}, evj[2] = {nullptr, nullptr};
  bool fused_timed = false, jacobi_timed = false;
  double fused_ms = 0.0, jacobi_ms = 0.0;
  int max_sweeps = kJacobiMaxSweeps;
  // L2 mode: per-block rank bytes, steps, budgets, errors; slice errors
  DevBuf l2rank, l2step, l2e2, l2berr, l2ovf, l2errp, l2cv, l2part, l2tgt;  // l2part: per-slice sums of squares
  DevBuf l2range, l2fpart;     // per-variable slice ranges, partial sums
  int l2_passes = 0;           // encode passes the last L2 call took
  // global-basis mode: bases, budgets, learning workspace, coefficients,
  // per-patch counts / exponents / slots, packed payload
  DevBuf gb_phi, gb_cv, gb_part, gb_tgt, gb_Q, gb_A0, gb_A1, gb_V, gb_norm, gb_alpha, gb_count, gb_kexp, gb_n0;
  DevBuf gb_slot, gb_nidx, gb_nraw, gb_idx_off, gb_raw_off, gb_idx, gb_q, gb_raw, gb_tot;
  int64_t gb_total = 0, gb_raw_bytes = 0;
  int gb_M = 0;
  double* gb_host = nullptr;        // pinned: sweep norms, payload totals
  // the device-driven encode sequence (Gram to encode) captured once per
  // layout and replayed; key: field, problem, buffers, model, knobs
  hipGraphExec_t dd_graph = nullptr;
  uint64_t dd_key[kDdKey] = {};
  bool dd_replayed = false;      // the last encode replayed the graph
  // one Jacobi sweep of the global basis (its rounds and the norm kernels)
  // captured once per workspace layout and replayed per sweep
  bool use_graphs = true;
  int64_t dd_max_items = 65536;     // device-driven launch up to this many slices
                                    // (looping encode workgroups measured slower
                                    // than one per slice above ~10^5 slices)
  hipStream_t gb_cap = nullptr;     // capture stream (default priority)
  hipGraphExec_t gb_sweep = nullptr;
  const void* gb_sweep_key[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  int gb_sweep_mp = 0;
  int64_t jacobi_sweeps = 0, jacobi_unconverged = 0;
  unsigned long long* jstats() { return reinterpret_cast<unsigned long long*>(counters.as<uint8_t>() + kJacobiAt); }
  PlanScratch* plan_scratch = nullptr;
  dls_model* model = nullptr;  // DLS_LEARNED
  int warm_iters = 2;
  int warm_margin = 1;
  DevBuf feat, zfeat, mlp_h1, mlp_h2, mlp_out, reject;
  int64_t nwarm_accept = 0, nwarm_reject = 0;
  void* pinned = nullptr;      // host staging for plan uploads
  size_t pinned_bytes = 0;
  uint8_t* hcnt = nullptr;     // pinned host copy of the counter block
  hipError_t host_counters() {
    if (hcnt) return hipSuccess;
    void* q = nullptr;
    hipError_t e = hipHostMalloc(&q, kCounterBytes, hipHostMallocDefault);
    if (e == hipSuccess) hcnt = static_cast<uint8_t*>(q);
    return e;
  }
  uint64_t esc_cap = 0;
  // results of the last dls_encode
  bool have_result = false;
  bool keep_coef = false;
  int64_t nesc = 0, nraw = 0, qv_bytes = 0, qa_bytes = 0;
  double gpu_ms = 0.0;
  ~dls_ctx() {
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
    for (auto& e : evs)
      if (e) (void)hipEventDestroy(e);
    for (int k = 0; k < 2; ++k) {
      if (evf[k]) (void)hipEventDestroy(evf[k]);
      if (evj[k]) (void)hipEventDestroy(evj[k]);
    }
    plan_scratch_delete(plan_scratch);
    if (pinned) (void)hipHostFree(pinned);
    if (hcnt) (void)hipHostFree(hcnt);
    if (hfused) (void)hipHostFree(hfused);
    if (gb_host) (void)hipHostFree(gb_host);
    if (gb_sweep) (void)hipGraphExecDestroy(gb_sweep);
    if (dd_graph) (void)hipGraphExecDestroy(dd_graph);
    if (gb_cap) (void)hipStreamDestroy(gb_cap);
  }
};

namespace {
// The plan's blocks split by size for the feature kernels (uploaded once per
// plan): at most kFeatSmall points, at most kWarmMaxPoints, larger.
dls_status feature_lists(dls_ctx* ctx, FeatureLists& L) {
  if (!ctx->feat_valid) {
    const auto& blocks = ctx->plan.blocks;
    std::vector<int32_t> l[3];
    for (size_t b = 0; b < blocks.size(); ++b)
      l[blocks[b].m <= kFeatSmall ? 0 : (blocks[b].m <= kWarmMaxPoints ? 1 : 2)].push_back(int32_t(b));
    std::vector<int32_t> all;
    all.reserve(blocks.size());
    for (int c = 0; c < 3; ++c) {
      ctx->feat_n[c] = int64_t(l[c].size());
      all.insert(all.end(), l[c].begin(), l[c].end());
    }
    HIP_TRY(ctx->feat_lists.ensure(std::max<size_t>(all.size(), 1) * sizeof(int32_t)));
    if (!all.empty())
      HIP_TRY(hipMemcpy(ctx->feat_lists.p, all.data(), all.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    ctx->feat_valid = true;
  }
  const int32_t* base = ctx->feat_lists.as<int32_t>();
  L = FeatureLists{base, ctx->feat_n[0], base + ctx->feat_n[0], ctx->feat_n[1],
                   base + ctx->feat_n[0] + ctx->feat_n[1], ctx->feat_n[2]};
  return DLS_OK;
}

// Eigen stage of a DLS_LEARNED encode: features, network forward (bf16),
// warm-started eigensolve, Jacobi on the rejected blocks.
dls_status learned_eigen(dls_ctx* ctx, const void* d_field, const Problem& p, const Dims& dims, hipStream_t s,
                         bool events = true) {
  dls_model* m = ctx->model;
  if (m == nullptr) return fail(DLS_EINVAL, "DLS_LEARNED without a model (dls_ctx_set_model)");
  if (m->device != ctx->device) return fail(DLS_EINVAL, "model lives on another device");
  const int64_t nb = int64_t(ctx->plan.blocks.size());
  unsigned long long* cnt = ctx->counters.as<unsigned long long>();
  HIP_TRY(ctx->feat.ensure(size_t(nb) * kNF * 4));
  HIP_TRY(ctx->mlp_out.ensure(size_t(nb) * kNO * 4));
  HIP_TRY(ctx->reject.ensure(size_t(nb)));
  FeatureLists fl;
  if (dls_status st = feature_lists(ctx, fl)) return st;
  HIP_TRY(launch_features(p.dtype, d_field, dims, ctx->desc.as<BlockDesc>(), fl, ctx->eps_v.as<double>(),
                          ctx->feat.as<float>(), s));
  if (dls_status st = model_infer(m, ctx->feat.as<float>(), nb, ctx->mlp_out.as<float>(), s)) return st;
  HIP_TRY(launch_warmstart(ctx->gram.as<double>(), ctx->item_start.as<int32_t>(), ctx->desc.as<BlockDesc>(), nb,
                           ctx->eps_v.as<double>(), p.r_max, ctx->mlp_out.as<float>(), ctx->warm_iters,
                           ctx->warm_margin, ctx->rank.as<uint8_t>(), ctx->lam.as<double>(), ctx->basis.as<double>(),
                           ctx->qv_size.as<int64_t>(), ctx->qa_size.as<int64_t>(), ctx->reject.as<uint8_t>(),
                           cnt + 2, ctx->jstats(), s));
  // the fallback Jacobi takes a compacted list of the rejected blocks, so its
  // workgroups are full of real work
  unsigned int* nrej = reinterpret_cast<unsigned int*>(reinterpret_cast<uint8_t*>(cnt) + kRejectCountAt);
  HIP_TRY(ctx->reject_list.ensure(size_t(nb) * sizeof(int32_t)));
  HIP_TRY(launch_compact_flags(ctx->reject.as<uint8_t>(), nb, ctx->reject_list.as<int32_t>(), nrej, s));
  if (events) HIP_TRY(hipEventRecord(ctx->evj[0], s));
  HIP_TRY(launch_eigen(16, ctx->gram.as<double>(), ctx->item_start.as<int32_t>(), ctx->desc.as<BlockDesc>(), nb,
                       ctx->eps_v.as<double>(), p.r_max, ctx->rank.as<uint8_t>(), ctx->lam.as<double>(),
                       ctx->basis.as<double>(), ctx->qv_size.as<int64_t>(), ctx->qa_size.as<int64_t>(), cnt + 1,
                       ctx->reject_list.as<int32_t>(), nrej, ctx->jstats(), ctx->max_sweeps, s));
  if (events) {
    HIP_TRY(hipEventRecord(ctx->evj[1], s));
    ctx->jacobi_timed = true;
  }
  return DLS_OK;
}
}  // namespace

namespace {

// The launches from the Gram to the classified rank lists, shared by both
// encode launches; `events` records the stage events (off while a graph is
// being captured).
dls_status enqueue_front(dls_ctx* ctx, const void* d_field, const Problem& p, const Dims& dims,
                         const GramSplit* split, hipStream_t s, bool events) {
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size()), ni = int64_t(pl.items.size());
  const int wp = p.wpad();
  unsigned long long* cnt = ctx->counters.as<unsigned long long>();
  HIP_TRY(launch_gram(wp, p.dtype, p.precision == DLS_PREC_BF16, d_field, dims, ctx->desc.as<BlockDesc>(),
                      ctx->items.as<Item>(), ni, split, ctx->gram.as<double>(), s));
  if (events) HIP_TRY(hipEventRecord(ctx->evs[0], s));
  // the warm start applies to blocks of at most kWarmMaxPoints points; a plan
  // without any takes the plain eigensolve directly
  if ((p.flags & DLS_LEARNED) && ctx->plan_warm_blocks > 0) {
    if (dls_status st = learned_eigen(ctx, d_field, p, dims, s, events)) return st;
  } else {
    if (events) HIP_TRY(hipEventRecord(ctx->evj[0], s));
    HIP_TRY(launch_eigen(wp, ctx->gram.as<double>(), ctx->item_start.as<int32_t>(), ctx->desc.as<BlockDesc>(),
                         nb, ctx->eps_v.as<double>(), p.r_max, ctx->rank.as<uint8_t>(), ctx->lam.as<double>(),
                         ctx->basis.as<double>(), ctx->qv_size.as<int64_t>(), ctx->qa_size.as<int64_t>(),
                         cnt + 1, nullptr, nullptr, ctx->jstats(), ctx->max_sweeps, s));
    if (events) {
      HIP_TRY(hipEventRecord(ctx->evj[1], s));
      ctx->jacobi_timed = true;
    }
  }
  if (events) HIP_TRY(hipEventRecord(ctx->evs[1], s));
  HIP_TRY(launch_scan(ctx->qv_size.as<int64_t>(), nb, ctx->qv_off.as<int64_t>(), ctx->scan_tmp.as<int64_t>(), s));
  HIP_TRY(launch_scan(ctx->qa_size.as<int64_t>(), nb, ctx->qa_off.as<int64_t>(), ctx->scan_tmp.as<int64_t>(), s));
  unsigned int* cls_count = reinterpret_cast<unsigned int*>(cnt + 4);
  HIP_TRY(launch_classify(ctx->items.as<Item>(), ni, ctx->rank.as<uint8_t>(),
                          split ? encode_small_limit(wp, p.dtype) : 0, cls_count, ctx->cls_lists.as<int32_t>(), s));
  if (events) HIP_TRY(hipEventRecord(ctx->evs[2], s));
  return DLS_OK;
}

// The device-driven encode: payload totals and one launch per rank class
// over the device-written class lists, into the payload buffers as sized.
dls_status enqueue_dd_encode(dls_ctx* ctx, const void* d_field, const Problem& p, const Dims& dims, hipStream_t s,
                             bool events) {
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size()), ni = int64_t(pl.items.size());
  const int wp = p.wpad();
  unsigned long long* cnt = ctx->counters.as<unsigned long long>();
  unsigned int* cls_count = reinterpret_cast<unsigned int*>(cnt + 4);
  unsigned int* overflow = reinterpret_cast<unsigned int*>(reinterpret_cast<uint8_t*>(cnt) + kOverflowAt);
  int64_t* totals = reinterpret_cast<int64_t*>(reinterpret_cast<uint8_t*>(cnt) + kTotalsAt);
  HIP_TRY(launch_totals(ctx->qv_off.as<int64_t>(), ctx->qv_size.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                        ctx->qa_size.as<int64_t>(), nb, totals, s));
  EscOut esc{cnt, ctx->esc_key.as<uint64_t>(), ctx->esc_val.as<uint64_t>(), ctx->esc_cap};
  if (events) HIP_TRY(hipEventRecord(ctx->evs[3], s));
  for (int c = 0; c < kEncodeClasses; ++c) {
    const EncodeWork work{cls_count + c, ni, int64_t(ctx->qv.n), int64_t(ctx->qa.n), overflow};
    HIP_TRY(launch_encode(wp, p.dtype, c, d_field, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(),
                          ctx->cls_lists.as<int32_t>() + int64_t(c) * ni, work, ctx->rank.as<uint8_t>(),
                          ctx->basis.as<double>(), ctx->qv_off.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                          ctx->code_off.as<int64_t>(), ctx->vconst.as<VarConst>(), ctx->qv.as<uint8_t>(),
                          ctx->qa.as<uint8_t>(), ctx->codes.as<uint8_t>(),
                          ctx->keep_coef ? ctx->coef.as<float>() : nullptr, esc, s));
  }
  return DLS_OK;
}

// What a captured device-driven sequence bakes in: every buffer address
// (through the allocation epoch), the field, the launch shapes, the model
// and the knobs (kDdKey words).
void dd_key(const dls_ctx* ctx, const void* d_field, const Problem& p, uint64_t key[kDdKey]) {
  const bool learned = (p.flags & DLS_LEARNED) != 0;
  key[0] = g_alloc_epoch.load();
  key[1] = uint64_t(reinterpret_cast<uintptr_t>(d_field));
  key[2] = uint64_t(p.flags) | (uint64_t(p.precision) << 8) | (uint64_t(p.dtype) << 12) | (uint64_t(p.r_max) << 16) |
           (uint64_t(p.wpad()) << 24) | (uint64_t(ctx->keep_coef) << 32) | (uint64_t(ctx->max_sweeps) << 40);
  key[3] = uint64_t(ctx->plan.blocks.size());
  key[4] = uint64_t(ctx->plan.items.size());
  key[5] = learned ? uint64_t(reinterpret_cast<uintptr_t>(ctx->model)) : 0;
  key[6] = learned && ctx->model ? ctx->model->version : 0;
  key[7] = uint64_t(ctx->warm_iters) | (uint64_t(ctx->warm_margin) << 16) | (uint64_t(ctx->plan_warm_blocks) << 32);
  key[8] = ctx->esc_cap;
  key[9] = uint64_t(ctx->split_nlarge);
  key[10] = uint64_t(ctx->split_nsmall);
  key[11] = uint64_t(ctx->feat_n[0]);
  key[12] = uint64_t(ctx->feat_n[1]);
  key[13] = uint64_t(ctx->feat_n[2]);
  key[14] = uint64_t(p.nx) ^ (uint64_t(p.ny) << 20) ^ (uint64_t(p.nz) << 40) ^ (uint64_t(p.nt) << 52);
  key[15] = uint64_t(p.px) | (uint64_t(p.py) << 8) | (uint64_t(p.pz) << 16) | (uint64_t(p.window) << 24) |
            (uint64_t(ctx->split_valid) << 32) | (uint64_t(ctx->feat_valid) << 33);
}

// Captures the device-driven sequence for the next calls with the same key
// (after an eager call, so every buffer and upload is in place).  A capture
// that fails leaves the eager launches in use.
void dd_capture(dls_ctx* ctx, const void* d_field, const Problem& p, const Dims& dims, const GramSplit* split) {
  if (ctx->dd_graph) {
    (void)hipGraphExecDestroy(ctx->dd_graph);
    ctx->dd_graph = nullptr;
  }
  if (ctx->gb_cap == nullptr && hipStreamCreateWithFlags(&ctx->gb_cap, hipStreamNonBlocking) != hipSuccess) {
    ctx->gb_cap = nullptr;
    (void)hipGetLastError();
    return;
  }
  uint64_t key[kDdKey];
  dd_key(ctx, d_field, p, key);
  if (hipStreamBeginCapture(ctx->gb_cap, hipStreamCaptureModeRelaxed) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  const std::string saved = g_err;
  dls_status st = enqueue_front(ctx, d_field, p, dims, split, ctx->gb_cap, false);
  if (st == DLS_OK) st = enqueue_dd_encode(ctx, d_field, p, dims, ctx->gb_cap, false);
  hipGraph_t g = nullptr;
  const hipError_t ce = hipStreamEndCapture(ctx->gb_cap, &g);
  g_err = saved;
  if (st != DLS_OK || ce != hipSuccess || g == nullptr) {
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
    return;
  }
  const hipError_t ie = hipGraphInstantiate(&ctx->dd_graph, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ie != hipSuccess) {
    ctx->dd_graph = nullptr;
    (void)hipGetLastError();
    return;
  }
  std::copy(key, key + kDdKey, ctx->dd_key);
}

// device time of the whole encode and of its five stages, from the events
dls_status finish_encode(dls_ctx* ctx) {
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
  ctx->gpu_ms = ms;
  const hipEvent_t marks[5][2] = {{ctx->evs[4], ctx->ev0}, {ctx->ev0, ctx->evs[0]}, {ctx->evs[0], ctx->evs[1]},
                                  {ctx->evs[1], ctx->evs[2]}, {ctx->evs[3], ctx->ev1}};
  for (int i = 0; i < 5; ++i) {
    HIP_TRY(hipEventElapsedTime(&ms, marks[i][0], marks[i][1]));
    ctx->stage_ms[i] = ms;
  }
  ctx->fused_ms = ctx->jacobi_ms = 0.0;
  if (ctx->fused_timed) {
    HIP_TRY(hipEventElapsedTime(&ms, ctx->evf[0], ctx->evf[1]));
    ctx->fused_ms = ms;
  }
  if (ctx->jacobi_timed) {
    HIP_TRY(hipEventElapsedTime(&ms, ctx->evj[0], ctx->evj[1]));
    ctx->jacobi_ms = ms;
  }
  // every path's last full readback of the counter block follows its Jacobi
  // (the global-basis mode counts its sweeps on the host)
  if (!(ctx->prob.flags & DLS_GLOBAL)) {
    unsigned long long js[1 + kJacobiSlots];
    std::memcpy(js, ctx->hcnt + kJacobiAt, sizeof(js));
    ctx->jacobi_unconverged = int64_t(js[0]);
    ctx->jacobi_sweeps = 0;
    for (int k = 1; k <= kJacobiSlots; ++k) ctx->jacobi_sweeps += int64_t(js[k]);
  }
  ctx->have_result = true;
  return DLS_OK;
}
}  // namespace

namespace {
// L2 / NRMSE-bounded encode (DLS_L2): the budget of every variable from its
// norm, Gram and eigensolve with the eigensolve bound sqrt(0.36 c_v), then
// encode passes until every block meets its budget (a failing block is
// raised one rank, or stored raw).  Payload offsets come from a device scan
// of the per-block sizes; every pass rewrites every block.
dls_status l2_encode(dls_ctx* ctx, const void* d_field, const Problem& p, const Dims& dims, hipStream_t s) {
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size()), ni = int64_t(pl.items.size());
  const int wp = p.wpad();
  unsigned long long* cnt = ctx->counters.as<unsigned long long>();
  HIP_TRY(ctx->l2rank.ensure(size_t(nb)));
  HIP_TRY(ctx->l2step.ensure(size_t(nb) * 8));
  HIP_TRY(ctx->l2e2.ensure(size_t(nb) * 8));
  HIP_TRY(ctx->l2berr.ensure(size_t(nb) * 8));
  HIP_TRY(ctx->l2ovf.ensure(size_t(nb)));
  HIP_TRY(ctx->l2errp.ensure(size_t(ni) * 8));
  HIP_TRY(ctx->l2cv.ensure(size_t(p.nvars) * 8));
  HIP_TRY(ctx->l2part.ensure(size_t(std::max<int64_t>(ni, 1)) * 8));
  // the targets were uploaded as the bounds; the eigensolve takes sqrt(0.36 c_v)
  HIP_TRY(ctx->l2tgt.ensure(size_t(p.nvars) * 8));
  HIP_TRY(hipMemcpyAsync(ctx->l2tgt.p, ctx->eps_v.p, size_t(p.nvars) * 8, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipEventRecord(ctx->ev0, s));
  // FP64 Gram whatever the precision: the rank test compares eigenvalue
  // tails with a share of e2 that is ~1e-8 of the energy at tight targets.
  // The same read gives every slice's finite sum of squares, so the budget
  // takes no pass of its own.
  HIP_TRY(launch_l2_gram(wp, p.dtype, d_field, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(), ni,
                         ctx->gram.as<double>(), ctx->l2part.as<double>(), s));
  {
    // each variable's slice range (blocks are variable-major)
    std::vector<int64_t> range(2 * size_t(p.nvars), 0);
    for (int64_t b = nb - 1; b >= 0; --b) range[2 * pl.blocks[b].var] = pl.item_start[b];
    for (int64_t b = 0; b < nb; ++b) range[2 * pl.blocks[b].var + 1] = pl.item_start[b + 1];
    HIP_TRY(ctx->l2range.ensure(range.size() * 8));
    HIP_TRY(ctx->l2fpart.ensure(size_t(p.nvars) * 256 * 8));
    HIP_TRY(hipMemcpyAsync(ctx->l2range.p, range.data(), range.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_l2_budget(ctx->l2part.as<double>(), ctx->l2range.as<int64_t>(), ctx->l2fpart.as<double>(),
                             ctx->l2tgt.as<double>(), p.nt * p.nx * p.ny * p.nz, p.nvars, ctx->l2cv.as<double>(),
                             ctx->eps_v.as<double>(), s));
    HIP_TRY(hipStreamSynchronize(s));  // the range vector is pageable host memory
  }
  HIP_TRY(hipEventRecord(ctx->evs[0], s));
  HIP_TRY(hipEventRecord(ctx->evj[0], s));
  HIP_TRY(launch_eigen(wp, ctx->gram.as<double>(), ctx->item_start.as<int32_t>(), ctx->desc.as<BlockDesc>(), nb,
                       ctx->eps_v.as<double>(), p.r_max, ctx->rank.as<uint8_t>(), ctx->lam.as<double>(),
                       ctx->basis.as<double>(), ctx->qv_size.as<int64_t>(), ctx->qa_size.as<int64_t>(), cnt + 1,
                       nullptr, nullptr, ctx->jstats(), ctx->max_sweeps, s));
  HIP_TRY(hipEventRecord(ctx->evj[1], s));
  ctx->jacobi_timed = true;
  HIP_TRY(hipEventRecord(ctx->evs[1], s));
  int64_t* totals = reinterpret_cast<int64_t*>(reinterpret_cast<uint8_t*>(cnt) + kTotalsAt);
  unsigned int* nfail = reinterpret_cast<unsigned int*>(reinterpret_cast<uint8_t*>(cnt) + kOverflowAt);
  HIP_TRY(ctx->host_counters());
  bool first = true;
  ctx->l2_passes = 0;
  for (int pass = 0; pass <= p.wpad() + 1; ++pass) {
    HIP_TRY(launch_l2_params(ctx->desc.as<BlockDesc>(), nb, ctx->lam.as<double>(), wp, ctx->rank.as<uint8_t>(),
                             ctx->l2cv.as<double>(), first, p.esize(), ctx->l2rank.as<uint8_t>(),
                             ctx->l2step.as<double>(), ctx->l2e2.as<double>(), ctx->qv_size.as<int64_t>(),
                             ctx->qa_size.as<int64_t>(), s));
    first = false;
    HIP_TRY(launch_scan(ctx->qv_size.as<int64_t>(), nb, ctx->qv_off.as<int64_t>(), ctx->scan_tmp.as<int64_t>(), s));
    HIP_TRY(launch_scan(ctx->qa_size.as<int64_t>(), nb, ctx->qa_off.as<int64_t>(), ctx->scan_tmp.as<int64_t>(), s));
    HIP_TRY(launch_totals(ctx->qv_off.as<int64_t>(), ctx->qv_size.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                          ctx->qa_size.as<int64_t>(), nb, totals, s));
    HIP_TRY(hipMemcpyAsync(ctx->hcnt, cnt, kCounterBytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    int64_t ht[2];
    std::memcpy(ht, ctx->hcnt + kTotalsAt, sizeof(ht));
    ctx->qv_bytes = ht[0];
    ctx->qa_bytes = ht[1];
    HIP_TRY(ctx->qv.ensure(size_t(std::max<int64_t>(ht[0], 16))));
    HIP_TRY(ctx->qa.ensure(size_t(std::max<int64_t>(ht[1], 16))));
    if (pass == 0) {
      HIP_TRY(hipEventRecord(ctx->evs[2], s));
      HIP_TRY(hipEventRecord(ctx->evs[3], s));
    }
    HIP_TRY(launch_zero(ctx->l2ovf.p, size_t(nb), s));
    HIP_TRY(launch_zero(nfail, sizeof(unsigned int), s));
    HIP_TRY(launch_l2_encode(wp, p.dtype, d_field, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(), ni,
                             ctx->l2rank.as<uint8_t>(), ctx->l2step.as<double>(), ctx->basis.as<double>(),
                             ctx->qv_off.as<int64_t>(), ctx->qa_off.as<int64_t>(), ctx->qv.as<uint8_t>(),
                             ctx->qa.as<uint8_t>(), ctx->l2ovf.as<uint8_t>(), ctx->l2errp.as<double>(), s));
    HIP_TRY(launch_l2_check(ctx->desc.as<BlockDesc>(), ctx->item_start.as<int32_t>(), nb, ctx->l2errp.as<double>(),
                            ctx->l2e2.as<double>(), ctx->l2ovf.as<uint8_t>(), p.r_max, ctx->l2rank.as<uint8_t>(),
                            ctx->l2berr.as<double>(), nfail, s));
    HIP_TRY(hipMemcpyAsync(ctx->hcnt, cnt, kCounterBytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    ++ctx->l2_passes;
    unsigned int hf;
    std::memcpy(&hf, ctx->hcnt + kOverflowAt, 4);
    if (hf == 0) break;
    if (pass == p.wpad() + 1) return fail(DLS_EDEVICE, "L2 encode did not settle");
  }
  HIP_TRY(hipEventRecord(ctx->ev1, s));
  // raw blocks, for the info
  std::vector<uint8_t> hr(static_cast<size_t>(nb));
  if (nb) HIP_TRY(hipMemcpy(hr.data(), ctx->l2rank.p, size_t(nb), hipMemcpyDeviceToHost));
  ctx->nraw = 0;
  for (uint8_t r : hr) ctx->nraw += r == kL2Raw ? 1 : 0;
  ctx->nesc = ctx->nesc_slots = 0;
  ctx->nwarm_accept = ctx->nwarm_reject = 0;
  ctx->nfast_accept = ctx->ndeferred = 0;
  ctx->launch_mode = 0;
  return DLS_OK;
}
}  // namespace

namespace {
// One Jacobi sweep of order Mp (Mp - 1 rounds, ending in A1) and its norm
// kernels (A1 copied back to A0, the off-diagonal and total sums of
// squares to out[0..1]).
hipError_t gb_sweep_launches(double* A0, double* A1, double* V, int Mp, double* part, double* out, hipStream_t s) {
  for (int r = 0; r < Mp - 1; ++r) {
    hipError_t e = launch_gb_jacobi_round((r & 1) ? A1 : A0, (r & 1) ? A0 : A1, V, Mp, r, s);
    if (e != hipSuccess) return e;
  }
  return launch_gb_offnorm(A1, A0, Mp, part, out, s);
}

// Runs one sweep on s: replays the captured graph of the current workspace
// (capturing it first when the buffers or the order changed), or launches
// the kernels one by one when graphs are off.
dls_status gb_sweep(dls_ctx* ctx, double* A0, double* A1, double* V, int Mp, double* part, double* out,
                    hipStream_t s) {
  if (!ctx->use_graphs) {
    HIP_TRY(gb_sweep_launches(A0, A1, V, Mp, part, out, s));
    return DLS_OK;
  }
  const void* key[6] = {A0, A1, V, part, out, nullptr};
  if (ctx->gb_sweep == nullptr || ctx->gb_sweep_mp != Mp || !std::equal(key, key + 6, ctx->gb_sweep_key)) {
    if (ctx->gb_sweep) {
      HIP_TRY(hipGraphExecDestroy(ctx->gb_sweep));
      ctx->gb_sweep = nullptr;
    }
    if (ctx->gb_cap == nullptr) HIP_TRY(hipStreamCreateWithFlags(&ctx->gb_cap, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(ctx->gb_cap, hipStreamCaptureModeThreadLocal));
    hipError_t le = gb_sweep_launches(A0, A1, V, Mp, part, out, ctx->gb_cap);
    hipGraph_t g = nullptr;
    hipError_t ce = hipStreamEndCapture(ctx->gb_cap, &g);
    if (le != hipSuccess || ce != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(DLS_EDEVICE, "capture of the Jacobi sweep failed");
    }
    hipError_t ie = hipGraphInstantiate(&ctx->gb_sweep, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(ie);
    std::copy(key, key + 6, ctx->gb_sweep_key);
    ctx->gb_sweep_mp = Mp;
  }
  HIP_TRY(hipGraphLaunch(ctx->gb_sweep, s));
  return DLS_OK;
}

// Global-basis encode (DLS_GLOBAL; Alg. 1 as the paper states it): the
// budget of every variable, then per variable its basis (learned by the
// parallel Jacobi on the FP64 Gram of the learning patches, or the cosine
// basis), then the coefficients of every patch-snapshot on the matrix
// cores, the per-patch selection with its exact check, and the packed
// payload.  One host round trip per Jacobi sweep (its convergence test)
// and one for the payload totals.
dls_status global_encode(dls_ctx* ctx, const void* d_field, const Problem& p, const Dims& dims, hipStream_t s) {
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size());
  const int M = p.px * p.py * p.pz, Mp = M + (M & 1);
  const int es = p.esize();
  ctx->gb_M = M;
  if (nb % p.nvars != 0) return fail(DLS_EDEVICE, "global plan is not variable-major");
  const int64_t nbv = nb / p.nvars;
  if (ctx->gb_host == nullptr) {
    void* q = nullptr;
    HIP_TRY(hipHostMalloc(&q, 64, hipHostMallocDefault));
    ctx->gb_host = static_cast<double*>(q);
  }
  HIP_TRY(ctx->gb_tgt.ensure(size_t(p.nvars) * 8));
  HIP_TRY(ctx->gb_cv.ensure(size_t(p.nvars) * 8));
  HIP_TRY(ctx->gb_part.ensure((size_t(p.nvars) * kGbSumParts + 2 * kGbParts) * 8));
  HIP_TRY(ctx->gb_norm.ensure(16));
  HIP_TRY(ctx->gb_tot.ensure(32));
  HIP_TRY(ctx->gb_phi.ensure(size_t(p.nvars) * M * M * 8));
  HIP_TRY(hipMemcpyAsync(ctx->gb_tgt.p, p.eps.data(), size_t(p.nvars) * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(ctx->ev0, s));
  HIP_TRY(launch_gb_budget(p.dtype, d_field, p.nt * p.nz * p.ny * p.nx, p.nvars, ctx->gb_tgt.as<double>(),
                           ctx->gb_part.as<double>(), ctx->gb_cv.as<double>(), s));
  // bases
  ctx->jacobi_sweeps = ctx->jacobi_unconverged = 0;
  HIP_TRY(hipEventRecord(ctx->evj[0], s));
  double* normpart = ctx->gb_part.as<double>() + size_t(p.nvars) * kGbSumParts;
  for (int v = 0; v < p.nvars; ++v) {
    double* phi = ctx->gb_phi.as<double>() + size_t(v) * M * M;
    if (p.basis == DLS_BASIS_COSINE) {
      HIP_TRY(launch_gb_cosine(p.px, p.py, p.pz, phi, s));
      continue;
    }
    const int64_t S = p.basis == DLS_BASIS_SVD ? 4 * int64_t(M) : M;
    HIP_TRY(ctx->gb_Q.ensure(size_t(S) * M * 8));
    HIP_TRY(ctx->gb_A0.ensure(size_t(Mp) * Mp * 8));
    HIP_TRY(ctx->gb_A1.ensure(size_t(Mp) * Mp * 8));
    HIP_TRY(ctx->gb_V.ensure(size_t(Mp) * Mp * 8));
    double *A0 = ctx->gb_A0.as<double>(), *A1 = ctx->gb_A1.as<double>(), *V = ctx->gb_V.as<double>();
    HIP_TRY(launch_gb_samples(p.dtype, d_field, dims, v, p.px, p.py, p.pz, p.basis, p.seed + uint64_t(v), S,
                              ctx->gb_Q.as<double>(), s));
    HIP_TRY(launch_gb_gram(ctx->gb_Q.as<double>(), S, M, Mp, A0, s));
    const double floor2 = (4e-16 * M) * (4e-16 * M);
    if (Mp <= 64) {
      // the whole eigensolve in one workgroup (A and V in LDS)
      HIP_TRY(launch_gb_jacobi_lds(A0, Mp, floor2, kGbMaxSweeps, A1, V, reinterpret_cast<int*>(ctx->gb_tot.p), s));
      HIP_TRY(hipMemcpyAsync(ctx->gb_host, ctx->gb_tot.p, 8, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      int inf2[2];
      std::memcpy(inf2, ctx->gb_host, 8);
      ctx->jacobi_sweeps += inf2[0];
      ctx->jacobi_unconverged += inf2[1];
      HIP_TRY(launch_gb_finish(A1, V, M, Mp, phi, s));
      continue;
    }
    HIP_TRY(launch_gb_eye(V, Mp, s));
    // sweeps of Mp - 1 rounds (odd, so each ends in A1; the norm kernel
    // copies it back to A0) until off(A) <= 4e-16 M ||A||_F (the rounding
    // floor of M^2 entries), or until a sweep leaves off(A) within 5 % of
    // the previous one (stalled at the floor; early sweeps can shrink it
    // by as little as a third, so only a stall counts)
    bool conv = false;
    int sweep = 0;
    double prev = HUGE_VAL;
    while (!conv && sweep < kGbMaxSweeps) {
      if (dls_status st = gb_sweep(ctx, A0, A1, V, Mp, normpart, ctx->gb_norm.as<double>(), s)) return st;
      HIP_TRY(hipMemcpyAsync(ctx->gb_host, ctx->gb_norm.p, 16, hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      ++sweep;
      const double off = ctx->gb_host[0], tot = ctx->gb_host[1];
      conv = off <= floor2 * tot || off >= 0.9 * prev;
      prev = off;
    }
    ctx->jacobi_sweeps += sweep;
    if (!conv) ++ctx->jacobi_unconverged;
    HIP_TRY(launch_gb_finish(A0, V, M, Mp, phi, s));
  }
  HIP_TRY(hipEventRecord(ctx->evj[1], s));
  ctx->jacobi_timed = true;
  HIP_TRY(hipEventRecord(ctx->evs[0], s));
  HIP_TRY(ctx->gb_count.ensure(size_t(nb) * 4));
  HIP_TRY(ctx->gb_kexp.ensure(size_t(nb) * 4));
  HIP_TRY(ctx->gb_n0.ensure(size_t(nb) * 4));
  HIP_TRY(ctx->gb_slot.ensure(size_t(nb) * 8 * M));
  if (M <= 64) {
    // one wave per patch-snapshot forms the coefficients and selects them
    HIP_TRY(hipEventRecord(ctx->evs[1], s));
    for (int v = 0; v < p.nvars; ++v)
      HIP_TRY(launch_gb_patch64(p.dtype, d_field, dims, ctx->desc.as<BlockDesc>(), v * nbv, (v + 1) * nbv,
                                ctx->gb_phi.as<double>() + size_t(v) * M * M, ctx->gb_cv.as<double>(), p.px, p.py, M,
                                ctx->gb_count.as<int32_t>(), ctx->gb_kexp.as<int32_t>(), ctx->gb_slot.as<uint8_t>(),
                                ctx->gb_n0.as<int32_t>(), s));
  } else {
    // coefficients on the matrix cores, one launch per variable (one basis
    // per launch), then one workgroup per patch-snapshot selects them
    HIP_TRY(ctx->gb_alpha.ensure(size_t(nb) * M * 8));
    for (int v = 0; v < p.nvars; ++v)
      HIP_TRY(launch_gb_project(p.dtype, d_field, dims, ctx->desc.as<BlockDesc>(), v * nbv, (v + 1) * nbv,
                                ctx->gb_phi.as<double>() + size_t(v) * M * M, p.px, p.py, M,
                                ctx->gb_alpha.as<double>(), s));
    HIP_TRY(hipEventRecord(ctx->evs[1], s));
    HIP_TRY(launch_gb_select(p.dtype, d_field, dims, ctx->desc.as<BlockDesc>(), nb, ctx->gb_phi.as<double>(),
                             ctx->gb_cv.as<double>(), ctx->gb_alpha.as<double>(), p.px, p.py, M,
                             ctx->gb_count.as<int32_t>(), ctx->gb_kexp.as<int32_t>(), ctx->gb_slot.as<uint8_t>(),
                             ctx->gb_n0.as<int32_t>(), s));
  }
  HIP_TRY(hipEventRecord(ctx->evs[2], s));
  HIP_TRY(hipEventRecord(ctx->evs[3], s));
  // packed payload: offsets of the kept coefficients and of the raw values
  HIP_TRY(ctx->gb_nidx.ensure(size_t(nb) * 8));
  HIP_TRY(ctx->gb_nraw.ensure(size_t(nb) * 8));
  HIP_TRY(ctx->gb_idx_off.ensure(size_t(nb) * 8));
  HIP_TRY(ctx->gb_raw_off.ensure(size_t(nb) * 8));
  HIP_TRY(ctx->scan_tmp.ensure(size_t(4 * (nb / 1024 + 4)) * sizeof(int64_t)));
  HIP_TRY(ctx->gb_tot.ensure(32));
  unsigned long long* raw_cnt = reinterpret_cast<unsigned long long*>(ctx->gb_tot.as<uint8_t>() + 16);
  HIP_TRY(launch_zero(raw_cnt, 8, s));
  HIP_TRY(launch_gb_sizes(ctx->desc.as<BlockDesc>(), nb, ctx->gb_count.as<int32_t>(), es,
                          ctx->gb_nidx.as<int64_t>(), ctx->gb_nraw.as<int64_t>(), raw_cnt, s));
  HIP_TRY(launch_scan(ctx->gb_nidx.as<int64_t>(), nb, ctx->gb_idx_off.as<int64_t>(), ctx->scan_tmp.as<int64_t>(), s));
  HIP_TRY(launch_scan(ctx->gb_nraw.as<int64_t>(), nb, ctx->gb_raw_off.as<int64_t>(), ctx->scan_tmp.as<int64_t>(), s));
  HIP_TRY(launch_totals(ctx->gb_idx_off.as<int64_t>(), ctx->gb_nidx.as<int64_t>(), ctx->gb_raw_off.as<int64_t>(),
                        ctx->gb_nraw.as<int64_t>(), nb, ctx->gb_tot.as<int64_t>(), s));
  HIP_TRY(hipMemcpyAsync(ctx->gb_host + 2, ctx->gb_tot.p, 24, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  int64_t tot[3];
  std::memcpy(tot, ctx->gb_host + 2, 24);
  ctx->gb_total = tot[0];
  ctx->gb_raw_bytes = tot[1];
  HIP_TRY(ctx->gb_idx.ensure(size_t(std::max<int64_t>(tot[0], 1)) * 2));
  HIP_TRY(ctx->gb_q.ensure(size_t(std::max<int64_t>(tot[0], 1)) * 4));
  HIP_TRY(ctx->gb_raw.ensure(size_t(std::max<int64_t>(tot[1], 1))));
  HIP_TRY(launch_gb_compact(ctx->desc.as<BlockDesc>(), nb, M, ctx->gb_count.as<int32_t>(), ctx->gb_slot.as<uint8_t>(),
                            ctx->gb_idx_off.as<int64_t>(), ctx->gb_raw_off.as<int64_t>(), es,
                            ctx->gb_idx.as<uint16_t>(), ctx->gb_q.as<int32_t>(), ctx->gb_raw.as<uint8_t>(), s));
  HIP_TRY(hipEventRecord(ctx->ev1, s));
  HIP_TRY(hipStreamSynchronize(s));
  ctx->nraw = tot[2];
  ctx->nesc = ctx->nesc_slots = 0;
  ctx->nwarm_accept = ctx->nwarm_reject = 0;
  ctx->nfast_accept = ctx->ndeferred = 0;
  ctx->launch_mode = 0;
  ctx->qv_bytes = 0;
  ctx->qa_bytes = 6 * tot[0] + tot[1];
  return DLS_OK;
}

void put_planes(std::vector<uint8_t>& out, const uint8_t* src, int64_t n, int nbytes) {
  for (int j = 0; j < nbytes; ++j)
    for (int64_t i = 0; i < n; ++i) out.push_back(src[i * nbytes + j]);
}

dls_status global_finalize(dls_ctx* ctx, uint8_t** out, size_t* out_bytes) {
  const Problem& p = ctx->prob;
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size());
  const int M = ctx->gb_M, es = p.esize();
  std::vector<int32_t> kexp(nb);
  std::vector<int64_t> ioff(nb), roff(nb);
  std::vector<uint16_t> idx(std::max<int64_t>(ctx->gb_total, 1));
  std::vector<int32_t> q(std::max<int64_t>(ctx->gb_total, 1));
  std::vector<uint8_t> raw(std::max<int64_t>(ctx->gb_raw_bytes, 1));
  std::vector<double> phi(size_t(p.nvars) * M * M), cv(p.nvars);
  if (nb) {
    HIP_TRY(hipMemcpy(kexp.data(), ctx->gb_kexp.p, nb * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(ioff.data(), ctx->gb_idx_off.p, nb * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(roff.data(), ctx->gb_raw_off.p, nb * 8, hipMemcpyDeviceToHost));
  }
  if (ctx->gb_total) {
    HIP_TRY(hipMemcpy(idx.data(), ctx->gb_idx.p, ctx->gb_total * 2, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(q.data(), ctx->gb_q.p, ctx->gb_total * 4, hipMemcpyDeviceToHost));
  }
  if (ctx->gb_raw_bytes) HIP_TRY(hipMemcpy(raw.data(), ctx->gb_raw.p, ctx->gb_raw_bytes, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(phi.data(), ctx->gb_phi.p, phi.size() * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(cv.data(), ctx->gb_cv.p, cv.size() * 8, hipMemcpyDeviceToHost));
  std::vector<int32_t> cnt(nb);
  if (nb) HIP_TRY(hipMemcpy(cnt.data(), ctx->gb_count.p, size_t(nb) * 4, hipMemcpyDeviceToHost));
  const int64_t npb = (nb + kBatchBlocks - 1) / kBatchBlocks;
  const int64_t nbatch = npb + p.nvars;
  std::vector<std::vector<uint8_t>> zs(nbatch);
  std::vector<uint64_t> usz(nbatch);
  std::atomic<bool> zfail{false};
  parallel_for(nbatch, [&](int64_t bi) {
    std::vector<uint8_t> rb;
    if (bi < npb) {
      const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks);
      std::vector<uint16_t> c16(b1 - b0);
      std::vector<int16_t> k16(b1 - b0);
      for (int64_t b = b0; b < b1; ++b) {
        c16[b - b0] = uint16_t(cnt[b]);
        k16[b - b0] = int16_t(kexp[b]);
      }
      put_planes(rb, reinterpret_cast<const uint8_t*>(c16.data()), b1 - b0, 2);
      put_planes(rb, reinterpret_cast<const uint8_t*>(k16.data()), b1 - b0, 2);
      int64_t i0 = b0 < nb ? ioff[b0] : 0, i1 = i0;
      for (int64_t b = b0; b < b1; ++b) i1 += cnt[b] == kGbRaw ? 0 : cnt[b];
      put_planes(rb, reinterpret_cast<const uint8_t*>(idx.data() + i0), i1 - i0, 2);
      std::vector<uint32_t> z(i1 - i0);
      for (int64_t i = i0; i < i1; ++i) z[i - i0] = (uint32_t(q[i]) << 1) ^ uint32_t(q[i] >> 31);
      put_planes(rb, reinterpret_cast<const uint8_t*>(z.data()), i1 - i0, 4);
      for (int64_t b = b0; b < b1; ++b)
        if (cnt[b] == kGbRaw) {
          const int64_t n = int64_t(pl.blocks[b].m) * es;
          rb.insert(rb.end(), raw.begin() + roff[b], raw.begin() + roff[b] + n);
        }
    } else {
      const int v = int(bi - npb);
      uint32_t hdr[2] = {uint32_t(p.basis), uint32_t(M)};
      const uint8_t* hp = reinterpret_cast<const uint8_t*>(hdr);
      rb.insert(rb.end(), hp, hp + 8);
      const uint8_t* cp = reinterpret_cast<const uint8_t*>(&cv[v]);
      rb.insert(rb.end(), cp, cp + 8);
      std::vector<uint32_t> z(size_t(M) * M);
      for (size_t i = 0; i < z.size(); ++i) {
        const int32_t qi = int32_t(std::nearbyint(phi[size_t(v) * M * M + i] * 16777216.0));
        z[i] = (uint32_t(qi) << 1) ^ uint32_t(qi >> 31);
      }
      put_planes(rb, reinterpret_cast<const uint8_t*>(z.data()), int64_t(z.size()), 4);
    }
    uLongf zn = compressBound(uLong(rb.size()));
    std::vector<uint8_t> zb(zn);
    if (compress2(zb.data(), &zn, rb.data(), uLong(rb.size()), kZlibLevel) != Z_OK) {
      zfail = true;
      return;
    }
    zb.resize(zn);
    zs[bi] = std::move(zb);
    usz[bi] = rb.size();
  });
  if (zfail) return fail(DLS_ENOMEM, "zlib compress2 failed");
  std::vector<StreamHeader::Batch> table(nbatch);
  uint64_t off = 0;
  for (int64_t i = 0; i < nbatch; ++i) {
    table[i] = StreamHeader::Batch{off, zs[i].size(), usz[i]};
    off += zs[i].size();
  }
  std::vector<uint8_t> hdr = write_header(p, nb, pl.bits, table, uint32_t(p.basis));
  const size_t total = hdr.size() + off;
  uint8_t* buf = static_cast<uint8_t*>(std::malloc(total ? total : 1));
  if (buf == nullptr) return fail(DLS_ENOMEM, "output allocation");
  std::memcpy(buf, hdr.data(), hdr.size());
  size_t pos = hdr.size();
  for (auto& z : zs) {
    std::memcpy(buf + pos, z.data(), z.size());
    pos += z.size();
  }
  *out = buf;
  *out_bytes = total;
  return DLS_OK;
}

// The patch-snapshot arrays of a global-basis stream, checked and moved into
// the device layout: counts, exponents, offsets of the kept coefficients and
// of the raw values, packed indices, coefficients, raw bytes, and the bases.
struct GlobalPayload {
  std::vector<int32_t> cnt, kexp;
  std::vector<int64_t> ioff, roff;
  std::vector<uint16_t> idx;
  std::vector<int32_t> q;
  std::vector<uint8_t> raw;
  std::vector<double> phi;
};

std::string global_unpack(const uint8_t* in, const StreamHeader& h, const Plan& pl, GlobalPayload& g) {
  const Problem& p = h.prob;
  const int64_t nb = h.nblocks;
  const int M = p.px * p.py * p.pz, es = p.esize();
  const int64_t npb = (nb + kBatchBlocks - 1) / kBatchBlocks;
  std::vector<std::vector<uint8_t>> raws(h.batches.size());
  std::vector<std::string> errs(h.batches.size());
  parallel_for(int64_t(h.batches.size()), [&](int64_t bi) {
    const auto& e = h.batches[bi];
    if (e.usize > (uint64_t(1) << 40)) {
      errs[bi] = "batch too large";
      return;
    }
    raws[bi].resize(e.usize);
    uLongf n = uLongf(e.usize);
    if (uncompress(raws[bi].data(), &n, in + h.header_bytes + e.off, uLong(e.csize)) != Z_OK || n != e.usize)
      errs[bi] = "zlib stream of a batch is corrupt";
  });
  for (auto& e : errs)
    if (!e.empty()) return e;
  g.cnt.resize(nb);
  g.kexp.resize(nb);
  g.ioff.resize(nb);
  g.roff.resize(nb);
  int64_t ti = 0, tr = 0;
  // first pass: counts and sizes
  for (int64_t bi = 0; bi < npb; ++bi) {
    const auto& r = raws[bi];
    const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks), n = b1 - b0;
    if (int64_t(r.size()) < 4 * n) return "batch payload truncated";
    int64_t kept = 0, rawb = 0;
    for (int64_t j = 0; j < n; ++j) {
      const int c = int(r[j]) | (int(r[n + j]) << 8);
      const int16_t k = int16_t(uint16_t(r[2 * n + j]) | (uint16_t(r[3 * n + j]) << 8));
      if (c != kGbRaw && c > M) return "coefficient count out of range";
      g.cnt[b0 + j] = c;
      g.kexp[b0 + j] = k;
      g.ioff[b0 + j] = ti + kept;
      g.roff[b0 + j] = tr + rawb;
      if (c == kGbRaw) rawb += int64_t(pl.blocks[b0 + j].m) * es;
      else kept += c;
    }
    if (int64_t(r.size()) != 4 * n + 6 * kept + rawb) return "batch size mismatch";
    ti += kept;
    tr += rawb;
  }
  g.idx.resize(std::max<int64_t>(ti, 1));
  g.q.resize(std::max<int64_t>(ti, 1));
  g.raw.resize(std::max<int64_t>(tr, 1));
  for (int64_t bi = 0; bi < npb; ++bi) {
    const auto& r = raws[bi];
    const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks), n = b1 - b0;
    const int64_t i0 = g.ioff[b0];
    int64_t kept = 0;
    for (int64_t b = b0; b < b1; ++b) kept += g.cnt[b] == kGbRaw ? 0 : g.cnt[b];
    const uint8_t* ip = r.data() + 4 * n;
    const uint8_t* qp = ip + 2 * kept;
    for (int64_t i = 0; i < kept; ++i) {
      g.idx[i0 + i] = uint16_t(ip[i] | (ip[kept + i] << 8));
      const uint32_t z = uint32_t(qp[i]) | (uint32_t(qp[kept + i]) << 8) | (uint32_t(qp[2 * kept + i]) << 16) |
                         (uint32_t(qp[3 * kept + i]) << 24);
      g.q[i0 + i] = int32_t(z >> 1) ^ -int32_t(z & 1);
    }
    for (int64_t b = b0; b < b1; ++b) {
      if (g.cnt[b] == kGbRaw) continue;
      for (int j = 0; j < g.cnt[b]; ++j) {
        const int s = g.idx[g.ioff[b] + j];
        if (s >= M || (j > 0 && s <= g.idx[g.ioff[b] + j - 1])) return "basis indices out of order";
      }
    }
    const uint8_t* rp = qp + 4 * kept;
    const int64_t rawb = int64_t(r.size()) - (rp - r.data());
    if (rawb > 0) std::memcpy(g.raw.data() + g.roff[b0], rp, size_t(rawb));
  }
  g.phi.resize(size_t(p.nvars) * M * M);
  for (int v = 0; v < p.nvars; ++v) {
    const auto& r = raws[npb + v];
    if (int64_t(r.size()) != 16 + 4 * int64_t(M) * M) return "basis batch size";
    uint32_t kind, mm;
    std::memcpy(&kind, r.data(), 4);
    std::memcpy(&mm, r.data() + 4, 4);
    if (int(mm) != M || kind != h.extra) return "basis batch header";
    const int64_t n = int64_t(M) * M;
    const uint8_t* zp = r.data() + 16;
    for (int64_t i = 0; i < n; ++i) {
      const uint32_t z = uint32_t(zp[i]) | (uint32_t(zp[n + i]) << 8) | (uint32_t(zp[2 * n + i]) << 16) |
                         (uint32_t(zp[3 * n + i]) << 24);
      g.phi[size_t(v) * n + i] = double(int32_t(z >> 1) ^ -int32_t(z & 1)) / 16777216.0;
    }
  }
  return "";
}

dls_status global_decompress(const uint8_t* in, const StreamHeader& h, const Plan& pl, void* d_out, hipStream_t s) {
  const Problem& p = h.prob;
  GlobalPayload g;
  std::string err = global_unpack(in, h, pl, g);
  if (!err.empty()) return fail(DLS_ECORRUPT, err);
  const int64_t nb = h.nblocks;
  const int M = p.px * p.py * p.pz;
  DevBuf desc, cnt, kexp, ioff, roff, idx, q, raw, phi;
  HIP_TRY(desc.ensure(size_t(nb) * sizeof(BlockDesc)));
  HIP_TRY(cnt.ensure(size_t(nb) * 4));
  HIP_TRY(kexp.ensure(size_t(nb) * 4));
  HIP_TRY(ioff.ensure(size_t(nb) * 8));
  HIP_TRY(roff.ensure(size_t(nb) * 8));
  HIP_TRY(idx.ensure(g.idx.size() * 2));
  HIP_TRY(q.ensure(g.q.size() * 4));
  HIP_TRY(raw.ensure(g.raw.size()));
  HIP_TRY(phi.ensure(g.phi.size() * 8));
  HIP_TRY(hipMemcpy(desc.p, pl.blocks.data(), size_t(nb) * sizeof(BlockDesc), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(cnt.p, g.cnt.data(), size_t(nb) * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(kexp.p, g.kexp.data(), size_t(nb) * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(ioff.p, g.ioff.data(), size_t(nb) * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(roff.p, g.roff.data(), size_t(nb) * 8, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(idx.p, g.idx.data(), g.idx.size() * 2, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(q.p, g.q.data(), g.q.size() * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(raw.p, g.raw.data(), g.raw.size(), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(phi.p, g.phi.data(), g.phi.size() * 8, hipMemcpyHostToDevice));
  const Dims dims{p.nx, p.ny, p.nz, p.nt};
  HIP_TRY(launch_gb_decode(p.dtype, d_out, dims, desc.as<BlockDesc>(), nb, p.nvars, phi.as<double>(), p.px, p.py, M,
                           cnt.as<int32_t>(), kexp.as<int32_t>(), ioff.as<int64_t>(), roff.as<int64_t>(),
                           idx.as<uint16_t>(), q.as<int32_t>(), raw.as<uint8_t>(), s));
  HIP_TRY(hipStreamSynchronize(s));
  return DLS_OK;
}
}  // namespace

namespace {
// The single-pass encode (DLS_PERSISTENT on plans of large FP32 blocks,
// W <= 16; reading R28): the Gram of every block's first slice gives a
// rank-1 basis (k_sketch_basis); one launch (k_fused) reads every slice once,
// encodes it with that basis, forms the slice's Gram partial, and the slice
// that completes its block verifies the basis on the whole Gram.  Blocks it
// does not verify take the Jacobi eigensolve and a device-driven encode that
// reads them again.  On success *done is set; otherwise (payload buffers too
// small, escape list full) the buffers are grown and the caller encodes the
// call again two-pass.
// Fraction of the blocks above which a predicted deferral makes the call run
// two-pass: on the 512^3 x 48 FP32 workload the single pass costs ~18 ms
// with every block verified and the deferred blocks' second read and
// device-driven encode ~23 ms more when all are deferred, against ~29 ms for
// the two-pass Gram + encode, so the two break even near one half.
constexpr double kFusedMaxPredictedDeferred = 0.5;

dls_status fused_encode(dls_ctx* ctx, const void* d_field, const Problem& p, const Dims& dims, hipStream_t s,
                        bool* done) {
  *done = false;
  ctx->fused_declined = false;
  ctx->npredicted = ctx->npruned = 0;
  if (int64_t(ctx->plan.items.size()) > int64_t(INT32_MAX)) return DLS_OK;  // one workgroup per slice
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size()), ni = int64_t(pl.items.size());
  unsigned long long* cnt = ctx->counters.as<unsigned long long>();
  if (!ctx->r1_valid) {  // static rank-1 payload offsets of the plan
    std::vector<int64_t> off(2 * size_t(nb));
    int64_t v = 0, a = 0;
    for (int64_t b = 0; b < nb; ++b) {
      off[b] = v;
      off[nb + b] = a;
      v += 4 * pad16(pl.blocks[b].w());
      a += 4 * pad16(pl.blocks[b].m);
    }
    HIP_TRY(ctx->r1_off.ensure(off.size() * sizeof(int64_t)));
    HIP_TRY(hipMemcpy(ctx->r1_off.p, off.data(), off.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    ctx->r1_valid = true;
  }
  // state: state[nb], deferred[nb] (u32 each), ndeferred (u32, padded), counters (u64)
  const size_t fbytes = 8 * size_t(nb) + 16 + kFusedNCounters * 8;
  HIP_TRY(ctx->fused.ensure(fbytes));
  uint8_t* fb = ctx->fused.as<uint8_t>();
  FusedState fs{reinterpret_cast<unsigned int*>(fb), reinterpret_cast<int32_t*>(fb + 4 * nb),
                reinterpret_cast<unsigned int*>(fb + 8 * nb), reinterpret_cast<unsigned long long*>(fb + 8 * nb + 16)};
  if (ctx->hfused == nullptr) {
    void* q = nullptr;
    HIP_TRY(hipHostMalloc(&q, 16 + kFusedNCounters * 8, hipHostMallocDefault));
    ctx->hfused = static_cast<unsigned long long*>(q);
  }
  // the rank-1 payload of every block is the least room needed
  HIP_TRY(ctx->qv.ensure(size_t(ctx->plan_qv_r1) + 16));
  HIP_TRY(ctx->qa.ensure(size_t(ctx->plan_qa_r1) + 16));
  if (ctx->keep_coef) HIP_TRY(ctx->coef.ensure(ctx->qa.n));
  HIP_TRY(launch_zero(fb, fbytes, s));
  const int wp = p.wpad();
  const bool bf16 = p.precision == DLS_PREC_BF16;
  EscOut esc{cnt, ctx->esc_key.as<uint64_t>(), ctx->esc_val.as<uint64_t>(), ctx->esc_cap};
  unsigned int* overflow = reinterpret_cast<unsigned int*>(reinterpret_cast<uint8_t*>(cnt) + kOverflowAt);
  unsigned int* cls_count = reinterpret_cast<unsigned int*>(cnt + 4);
  // the sketch: Gram partials of every block's first slice (item_start[b]
  // is that slice), then its rank-1 basis
  const GramSplit first{ctx->item_start.as<int32_t>(), nb, nullptr, 0};
  HIP_TRY(launch_gram(wp, p.dtype, bf16, d_field, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(), ni, &first,
                      ctx->gram.as<double>(), s));
  HIP_TRY(launch_sketch_basis(ctx->gram.as<double>(), ctx->item_start.as<int32_t>(), ctx->items.as<Item>(),
                              ctx->desc.as<BlockDesc>(), nb, ctx->eps_v.as<double>(), ctx->r1_off.as<int64_t>(),
                              ctx->rank.as<uint8_t>(), ctx->lam.as<double>(), ctx->basis.as<double>(),
                              ctx->qv_size.as<int64_t>(), ctx->qa_size.as<int64_t>(), ctx->qv_off.as<int64_t>(),
                              ctx->qa_off.as<int64_t>(), fs.state, fs.counters, s));
  // the sketch's prediction decides the form: a deferred block costs the
  // single pass a second read and encode, so when more than a fraction of the
  // blocks is predicted to fail verification the call runs two-pass
  HIP_TRY(hipMemcpyAsync(ctx->hfused + 2, fs.counters, kFusedNCounters * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  ctx->npredicted = int64_t(ctx->hfused[2 + kFusedLikely]);
  ctx->npruned = int64_t(ctx->hfused[2 + kFusedPruned]);
  if (double(ctx->npredicted) > kFusedMaxPredictedDeferred * double(nb)) {
    ctx->fused_declined = true;
    return DLS_OK;
  }
  HIP_TRY(hipEventRecord(ctx->evf[0], s));
  HIP_TRY(launch_fused(bf16, static_cast<const float*>(d_field), dims,
                       ctx->desc.as<BlockDesc>(),
                       ctx->items.as<Item>(), ni, ctx->vconst.as<VarConst>(), ctx->gram.as<double>(), fs.state,
                       ctx->basis.as<double>(), ctx->qv_off.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                       ctx->code_off.as<int64_t>(), ctx->qv.as<uint8_t>(), ctx->qa.as<uint8_t>(),
                       ctx->codes.as<uint8_t>(), ctx->keep_coef ? ctx->coef.as<float>() : nullptr, esc, s));
  HIP_TRY(hipEventRecord(ctx->evf[1], s));
  ctx->fused_timed = true;
  HIP_TRY(hipEventRecord(ctx->evs[0], s));
  HIP_TRY(launch_verify(ctx->gram.as<double>(), ctx->item_start.as<int32_t>(), ctx->desc.as<BlockDesc>(), nb,
                        ctx->eps_v.as<double>(), ctx->basis.as<double>(), ctx->lam.as<double>(), fs, s));
  // deferred blocks: Jacobi, payload regions after the rank-1 ones, their
  // slices encoded device-driven
  HIP_TRY(hipEventRecord(ctx->evj[0], s));
  HIP_TRY(launch_eigen(wp, ctx->gram.as<double>(), ctx->item_start.as<int32_t>(), ctx->desc.as<BlockDesc>(), nb,
                       ctx->eps_v.as<double>(), p.r_max, ctx->rank.as<uint8_t>(), ctx->lam.as<double>(),
                       ctx->basis.as<double>(), ctx->qv_size.as<int64_t>(), ctx->qa_size.as<int64_t>(), cnt + 1,
                       fs.deferred, fs.ndeferred, ctx->jstats(), ctx->max_sweeps, s));
  HIP_TRY(hipEventRecord(ctx->evj[1], s));
  ctx->jacobi_timed = true;
  HIP_TRY(hipEventRecord(ctx->evs[1], s));
  HIP_TRY(launch_alloc_deferred(fs.deferred, fs.ndeferred, nb, ctx->qv_size.as<int64_t>(), ctx->qa_size.as<int64_t>(),
                                fs.counters, ctx->plan_qv_r1, ctx->plan_qa_r1, ctx->qv_off.as<int64_t>(),
                                ctx->qa_off.as<int64_t>(), s));
  HIP_TRY(launch_classify(ctx->items.as<Item>(), ni, ctx->rank.as<uint8_t>(), 0, cls_count,
                          ctx->cls_lists.as<int32_t>(), s, fs.state));
  HIP_TRY(hipEventRecord(ctx->evs[2], s));
  HIP_TRY(hipEventRecord(ctx->evs[3], s));
  for (int c = 0; c < kRankClasses; ++c) {
    const EncodeWork work{cls_count + c, ni, int64_t(ctx->qv.n), int64_t(ctx->qa.n), overflow};
    HIP_TRY(launch_encode(wp, p.dtype, c, d_field, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(),
                          ctx->cls_lists.as<int32_t>() + int64_t(c) * ni, work, ctx->rank.as<uint8_t>(),
                          ctx->basis.as<double>(), ctx->qv_off.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                          ctx->code_off.as<int64_t>(), ctx->vconst.as<VarConst>(), ctx->qv.as<uint8_t>(),
                          ctx->qa.as<uint8_t>(), ctx->codes.as<uint8_t>(),
                          ctx->keep_coef ? ctx->coef.as<float>() : nullptr, esc, s));
  }
  HIP_TRY(launch_fix_escapes(ctx->esc_key.as<uint64_t>(), cnt, ctx->esc_cap, fs.state,
                             fs.counters + kFusedDropped, s));
  // rank-class lists of every slice, for the device decode of this result
  HIP_TRY(launch_zero(cls_count, kEncodeClasses * sizeof(unsigned int), s));
  HIP_TRY(launch_classify(ctx->items.as<Item>(), ni, ctx->rank.as<uint8_t>(), 0, cls_count,
                          ctx->cls_lists.as<int32_t>(), s, nullptr));
  HIP_TRY(hipEventRecord(ctx->ev1, s));
  HIP_TRY(ctx->host_counters());
  HIP_TRY(hipMemcpyAsync(ctx->hcnt, cnt, kCounterBytes, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipMemcpyAsync(ctx->hfused, fb + 8 * nb, 16 + kFusedNCounters * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  unsigned long long hc[4];
  unsigned int hov;
  std::memcpy(hc, ctx->hcnt, sizeof(hc));
  std::memcpy(&hov, ctx->hcnt + kOverflowAt, 4);
  unsigned int ndef;
  std::memcpy(&ndef, ctx->hfused, 4);
  const unsigned long long* fc = ctx->hfused + 2;
  ctx->nesc_slots = int64_t(hc[0]);
  ctx->nesc = int64_t(hc[0] - fc[kFusedDropped]);
  ctx->nraw = int64_t(hc[1]);
  ctx->qv_bytes = ctx->plan_qv_r1 + int64_t(fc[kFusedQvCursor]);
  ctx->qa_bytes = ctx->plan_qa_r1 + int64_t(fc[kFusedQaCursor]);
  ctx->nfast_accept = int64_t(fc[kFusedAccepted]);
  ctx->ndeferred = int64_t(ndef);
  const bool fits = hov == 0 && hc[0] <= ctx->esc_cap && ctx->qv_bytes <= int64_t(ctx->qv.n) &&
                    ctx->qa_bytes <= int64_t(ctx->qa.n);
  if (fits) {
    *done = true;
    ctx->launch_mode = 2;
    ctx->nwarm_accept = 0;  // no block of these plans is small enough for the warm start
    ctx->nwarm_reject = (p.flags & DLS_LEARNED) ? nb : 0;
    return DLS_OK;
  }
  // grow with headroom for later calls; the caller encodes this call two-pass
  HIP_TRY(ctx->qv.grow(size_t(ctx->qv_bytes + ctx->qv_bytes / 4 + 16)));
  HIP_TRY(ctx->qa.grow(size_t(ctx->qa_bytes + ctx->qa_bytes / 4 + 16)));
  if (ctx->keep_coef) HIP_TRY(ctx->coef.grow(ctx->qa.n));
  if (hc[0] > ctx->esc_cap) {
    ctx->esc_cap = hc[0] + (hc[0] >> 3) + 1024;
    HIP_TRY(ctx->esc_key.ensure(ctx->esc_cap * 8));
    HIP_TRY(ctx->esc_val.ensure(ctx->esc_cap * 8));
  }
  HIP_TRY(launch_zero(cnt, kCounterBytes, s));
  return DLS_OK;
}
}  // namespace

namespace {
// Host half of an L2-mode encode: per batch of 1000 blocks the rank bytes,
// the steps, the qV and qA planes and the raw blocks' values, deflated.
dls_status l2_finalize(dls_ctx* ctx, uint8_t** out, size_t* out_bytes) {
  const Problem& p = ctx->prob;
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size());
  std::vector<uint8_t> rank(nb), qv(std::max<int64_t>(ctx->qv_bytes, 1)), qa(std::max<int64_t>(ctx->qa_bytes, 1));
  std::vector<double> step(nb);
  std::vector<int64_t> qv_off(nb), qa_off(nb);
  if (nb) {
    HIP_TRY(hipMemcpy(rank.data(), ctx->l2rank.p, nb, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(step.data(), ctx->l2step.p, nb * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(qv_off.data(), ctx->qv_off.p, nb * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(qa_off.data(), ctx->qa_off.p, nb * 8, hipMemcpyDeviceToHost));
  }
  if (ctx->qv_bytes) HIP_TRY(hipMemcpy(qv.data(), ctx->qv.p, ctx->qv_bytes, hipMemcpyDeviceToHost));
  if (ctx->qa_bytes) HIP_TRY(hipMemcpy(qa.data(), ctx->qa.p, ctx->qa_bytes, hipMemcpyDeviceToHost));
  const int64_t nbatch = (nb + kBatchBlocks - 1) / kBatchBlocks;
  const int es = p.esize();
  std::vector<std::vector<uint8_t>> zs(nbatch);
  std::vector<uint64_t> usz(nbatch);
  std::atomic<bool> zfail{false};
  parallel_for(nbatch, [&](int64_t bi) {
    const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks);
    std::vector<uint8_t> raw;
    raw.insert(raw.end(), rank.begin() + b0, rank.begin() + b1);
    const uint8_t* sp = reinterpret_cast<const uint8_t*>(step.data() + b0);
    raw.insert(raw.end(), sp, sp + 8 * (b1 - b0));
    for (int64_t b = b0; b < b1; ++b) {
      const int r = rank[b] == kL2Raw ? 0 : rank[b];
      const int64_t n = int64_t(pl.blocks[b].w()) * r, pad = pad16(n);
      for (int j = 0; j < 4; ++j) {
        const uint8_t* src = qv.data() + qv_off[b] + j * pad;
        raw.insert(raw.end(), src, src + n);
      }
    }
    for (int64_t b = b0; b < b1; ++b) {
      const int r = rank[b] == kL2Raw ? 0 : rank[b];
      const int64_t n = int64_t(pl.blocks[b].m) * r, pad = pad16(n);
      for (int j = 0; j < 4; ++j) {
        const uint8_t* src = qa.data() + qa_off[b] + j * pad;
        raw.insert(raw.end(), src, src + n);
      }
    }
    for (int64_t b = b0; b < b1; ++b) {
      if (rank[b] != kL2Raw) continue;
      const int64_t n = int64_t(pl.blocks[b].w()) * pl.blocks[b].m * es;
      const uint8_t* src = qa.data() + qa_off[b];
      raw.insert(raw.end(), src, src + n);
    }
    uLongf zn = compressBound(uLong(raw.size()));
    std::vector<uint8_t> z(zn);
    if (compress2(z.data(), &zn, raw.data(), uLong(raw.size()), kZlibLevel) != Z_OK) {
      zfail = true;
      return;
    }
    z.resize(zn);
    zs[bi] = std::move(z);
    usz[bi] = raw.size();
  });
  if (zfail) return fail(DLS_ENOMEM, "zlib compress2 failed");
  std::vector<StreamHeader::Batch> table(nbatch);
  uint64_t off = 0;
  for (int64_t i = 0; i < nbatch; ++i) {
    table[i] = StreamHeader::Batch{off, zs[i].size(), usz[i]};
    off += zs[i].size();
  }
  std::vector<uint8_t> hdr = write_header(p, nb, pl.bits, table);
  const size_t total = hdr.size() + off;
  uint8_t* buf = static_cast<uint8_t*>(std::malloc(total ? total : 1));
  if (buf == nullptr) return fail(DLS_ENOMEM, "output allocation");
  std::memcpy(buf, hdr.data(), hdr.size());
  size_t pos = hdr.size();
  for (auto& z : zs) {
    std::memcpy(buf + pos, z.data(), z.size());
    pos += z.size();
  }
  *out = buf;
  *out_bytes = total;
  return DLS_OK;
}

// One inflated L2-mode batch moved into the device layout (the encoder's
// padding rules) at the given per-block offsets; "" on success.
std::string l2_unpack_batch(const uint8_t* in, const StreamHeader& h, const Plan& pl, int64_t bi,
                            std::vector<uint8_t>& rank, std::vector<double>& step, const std::vector<int64_t>& qv_off,
                            const std::vector<int64_t>& qa_off, std::vector<uint8_t>& qv, std::vector<uint8_t>& qa) {
  const auto& e = h.batches[bi];
  if (e.usize > (uint64_t(1) << 40)) return "batch too large";
  std::vector<uint8_t> raw(e.usize);
  uLongf n = uLongf(e.usize);
  if (uncompress(raw.data(), &n, in + h.header_bytes + e.off, uLong(e.csize)) != Z_OK || n != e.usize)
    return "zlib stream of a batch is corrupt";
  const int64_t nb = int64_t(pl.blocks.size());
  const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks);
  const int es = h.prob.esize();
  size_t pos = size_t(9 * (b1 - b0));
  if (pos > raw.size()) return "batch payload truncated";
  for (int64_t b = b0; b < b1; ++b) {
    if (rank[b] != raw[b - b0]) return "rank table mismatch";
    std::memcpy(&step[b], raw.data() + (b1 - b0) + 8 * (b - b0), 8);
  }
  for (int pass = 0; pass < 3; ++pass)
    for (int64_t b = b0; b < b1; ++b) {
      const BlockDesc& d = pl.blocks[b];
      const int r = rank[b] == kL2Raw ? 0 : rank[b];
      if (pass == 2) {
        if (rank[b] != kL2Raw) continue;
        const size_t nbytes = size_t(d.w()) * d.m * es;
        if (pos + nbytes > raw.size()) return "batch payload truncated";
        std::memcpy(qa.data() + qa_off[b], raw.data() + pos, nbytes);
        pos += nbytes;
        continue;
      }
      const int64_t cnt = int64_t(pass == 0 ? d.w() : d.m) * r, pad = pad16(cnt);
      std::vector<uint8_t>& dst = pass == 0 ? qv : qa;
      const int64_t base = pass == 0 ? qv_off[b] : qa_off[b];
      for (int j = 0; j < 4; ++j) {
        if (pos + size_t(cnt) > raw.size()) return "batch payload truncated";
        std::memcpy(dst.data() + base + j * pad, raw.data() + pos, size_t(cnt));
        pos += size_t(cnt);
      }
    }
  if (pos != raw.size()) return "batch payload size mismatch";
  return "";
}

// dls_decompress of an L2-mode stream: ranks first (sizes, offsets), then
// every batch into the device layout, then the decode kernel.
dls_status l2_decompress(const uint8_t* in, const StreamHeader& h, const Plan& pl, void* d_out, hipStream_t s) {
  const Problem& p = h.prob;
  const int64_t nb = h.nblocks, nbatch = int64_t(h.batches.size());
  std::vector<uint8_t> rank(nb);
  std::vector<double> step(nb);
  std::vector<std::string> errs(nbatch);
  // the rank bytes lead each batch: inflate once for them
  parallel_for(nbatch, [&](int64_t bi) {
    const auto& e = h.batches[bi];
    if (e.usize > (uint64_t(1) << 40)) { errs[bi] = "batch too large"; return; }
    std::vector<uint8_t> raw(e.usize);
    uLongf n = uLongf(e.usize);
    if (uncompress(raw.data(), &n, in + h.header_bytes + e.off, uLong(e.csize)) != Z_OK || n != e.usize) {
      errs[bi] = "zlib stream of a batch is corrupt";
      return;
    }
    const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks);
    if (raw.size() < size_t(b1 - b0)) { errs[bi] = "batch payload truncated"; return; }
    for (int64_t b = b0; b < b1; ++b) rank[b] = raw[b - b0];
  });
  for (auto& e : errs)
    if (!e.empty()) return fail(DLS_ECORRUPT, e);
  std::vector<int64_t> qv_off(nb), qa_off(nb);
  int64_t qv_bytes = 0, qa_bytes = 0;
  const int es = p.esize();
  for (int64_t b = 0; b < nb; ++b) {
    const BlockDesc& d = pl.blocks[b];
    const int r = rank[b];
    if (r != kL2Raw && r > std::min(p.r_max, d.w())) return fail(DLS_ECORRUPT, "rank out of range");
    qv_off[b] = qv_bytes;
    qa_off[b] = qa_bytes;
    if (r == kL2Raw) {
      qa_bytes += pad16(int64_t(d.w()) * d.m * es);
    } else {
      qv_bytes += 4 * pad16(int64_t(d.w()) * r);
      qa_bytes += 4 * pad16(int64_t(d.m) * r);
    }
  }
  std::vector<uint8_t> qv(std::max<int64_t>(qv_bytes, 1)), qa(std::max<int64_t>(qa_bytes, 1));
  parallel_for(nbatch, [&](int64_t bi) { errs[bi] = l2_unpack_batch(in, h, pl, bi, rank, step, qv_off, qa_off, qv, qa); });
  for (auto& e : errs)
    if (!e.empty()) return fail(DLS_ECORRUPT, e);
  const Dims dims{p.nx, p.ny, p.nz, p.nt};
  DevBuf d_desc, d_items, d_rank, d_step, d_qvo, d_qao, d_qv, d_qa;
  HIP_TRY(d_desc.ensure(pl.blocks.size() * sizeof(BlockDesc)));
  HIP_TRY(d_items.ensure(pl.items.size() * sizeof(Item)));
  HIP_TRY(d_rank.ensure(nb));
  HIP_TRY(d_step.ensure(nb * 8));
  HIP_TRY(d_qvo.ensure(nb * 8));
  HIP_TRY(d_qao.ensure(nb * 8));
  HIP_TRY(d_qv.ensure(qv.size()));
  HIP_TRY(d_qa.ensure(qa.size()));
  HIP_TRY(hipMemcpyAsync(d_desc.p, pl.blocks.data(), pl.blocks.size() * sizeof(BlockDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_items.p, pl.items.data(), pl.items.size() * sizeof(Item), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_rank.p, rank.data(), nb, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_step.p, step.data(), nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qvo.p, qv_off.data(), nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qao.p, qa_off.data(), nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qv.p, qv.data(), qv.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qa.p, qa.data(), qa.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_l2_decode(p.wpad(), p.dtype, d_out, dims, d_desc.as<BlockDesc>(), d_items.as<Item>(),
                           int64_t(pl.items.size()), d_rank.as<uint8_t>(), d_step.as<double>(), d_qvo.as<int64_t>(),
                           d_qao.as<int64_t>(), d_qv.as<uint8_t>(), d_qa.as<uint8_t>(), s));
  HIP_TRY(hipStreamSynchronize(s));
  return DLS_OK;
}
}  // namespace

extern "C" {

const char* dls_last_error(void) { return g_err.c_str(); }

void dls_free(void* p) { std::free(p); }

dls_status dls_ctx_create(int device, dls_ctx** out) {
  if (out == nullptr) return fail(DLS_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DLS_EINVAL, "no such device");
  std::unique_ptr<dls_ctx> c(new (std::nothrow) dls_ctx());
  if (!c) return fail(DLS_ENOMEM, "context allocation");
  c->device = device;
  HIP_TRY(hipSetDevice(device));
  HIP_TRY(hipEventCreate(&c->ev0));
  HIP_TRY(hipEventCreate(&c->ev1));
  for (auto& e : c->evs) HIP_TRY(hipEventCreate(&e));
  for (int k = 0; k < 2; ++k) {
    HIP_TRY(hipEventCreate(&c->evf[k]));
    HIP_TRY(hipEventCreate(&c->evj[k]));
  }
  c->plan_scratch = plan_scratch_new();
  *out = c.release();
  return DLS_OK;
}

dls_status dls_ctx_set_launch(dls_ctx* ctx, int64_t device_driven_max_items) {
  if (ctx == nullptr || device_driven_max_items < 0) return fail(DLS_EINVAL, "bad argument");
  ctx->dd_max_items = device_driven_max_items;
  return DLS_OK;
}

dls_status dls_ctx_set_graphs(dls_ctx* ctx, int enabled) {
  if (ctx == nullptr || (enabled != 0 && enabled != 1)) return fail(DLS_EINVAL, "bad argument");
  ctx->use_graphs = enabled != 0;
  return DLS_OK;
}

dls_status dls_ctx_set_jacobi_sweeps(dls_ctx* ctx, int max_sweeps) {
  if (ctx == nullptr) return fail(DLS_EINVAL, "ctx is NULL");
  if (max_sweeps < 1 || max_sweeps > 64) return fail(DLS_EINVAL, "max_sweeps must lie in [1, 64]");
  ctx->max_sweeps = max_sweeps;
  return DLS_OK;
}

void dls_ctx_destroy(dls_ctx* ctx) {
  if (ctx == nullptr) return;
  (void)hipSetDevice(ctx->device);
  delete ctx;
}

dls_status dls_encode(dls_ctx* ctx, const void* d_field, const dls_params* params, void* stream,
                      int keep_coef) {
  if (ctx == nullptr) return fail(DLS_EINVAL, "ctx is NULL");
  if (d_field == nullptr) return fail(DLS_EINVAL, "field is NULL");
  Problem p;
  if (dls_status s = validate(params, p)) return s;
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(hipSetDevice(ctx->device));
  ctx->have_result = false;
  ctx->fused_timed = ctx->jacobi_timed = false;
  ctx->fused_declined = false;
  ctx->npredicted = ctx->npruned = 0;
  HIP_TRY(hipEventRecord(ctx->evs[4], s));
  const bool adaptive = (p.flags & DLS_ADAPTIVE) != 0;
  if (adaptive) {
    // the adaptive plan depends on snapshot 0, so it is recomputed on every
    // call; the block list is expanded and uploaded again only when the new
    // split bits differ from those of the resident plan
    Plan fresh;
    std::string err;
    hipError_t he = adaptive_plan(p, d_field, s, *ctx->plan_scratch, fresh, err);
    if (he != hipSuccess) return fail(he == hipErrorOutOfMemory ? DLS_ENOMEM : DLS_EDEVICE, "adaptive plan: " + err);
    if (!(ctx->plan_valid && same_layout(ctx->prob, p) && fresh.bits == ctx->plan.bits)) {
      ctx->plan_valid = false;
      ctx->plan = std::move(fresh);
    }
  }

  // plan: uniform tiling depends on the problem statement only, so it is cached
  const auto th0 = std::chrono::steady_clock::now();
  if (!ctx->plan_valid || !same_layout(ctx->prob, p)) {
    ctx->plan_valid = false;
    if (!adaptive) {
      ctx->plan = Plan();
      ctx->plan.leaves.assign(p.nvars, uniform_leaves(p));
      ctx->plan.bits.assign(p.nvars, {});
    }
    build_blocks(p, ctx->plan, slice_points(p));
    ctx->split_valid = false;
    ctx->feat_valid = false;
    ctx->plan_warm_blocks = 0;
    ctx->r1_valid = false;
    ctx->plan_min_points = ctx->plan.blocks.empty() ? 0 : INT64_MAX;
    ctx->plan_qv_r1 = ctx->plan_qa_r1 = 0;
    for (const BlockDesc& d : ctx->plan.blocks) {
      ctx->plan_warm_blocks += d.m <= kWarmMaxPoints ? 1 : 0;
      ctx->plan_min_points = std::min<int64_t>(ctx->plan_min_points, d.m);
      ctx->plan_qv_r1 += 4 * pad16(d.w());
      ctx->plan_qa_r1 += 4 * pad16(d.m);
    }
    if (ctx->plan.blocks.size() >= (size_t(1) << 31)) return fail(DLS_EINVAL, "too many blocks");
    const Plan& pl = ctx->plan;
    HIP_TRY(ctx->desc.ensure(pl.blocks.size() * sizeof(BlockDesc)));
    HIP_TRY(ctx->items.ensure(pl.items.size() * sizeof(Item)));
    HIP_TRY(ctx->item_start.ensure(pl.item_start.size() * sizeof(int32_t)));
    HIP_TRY(ctx->code_off.ensure(pl.code_off.size() * sizeof(int64_t)));
    // one pinned staging buffer for the four plan arrays, then async copies
    const size_t sz[4] = {pl.blocks.size() * sizeof(BlockDesc), pl.items.size() * sizeof(Item),
                          pl.item_start.size() * sizeof(int32_t), pl.code_off.size() * sizeof(int64_t)};
    const void* src[4] = {pl.blocks.data(), pl.items.data(), pl.item_start.data(), pl.code_off.data()};
    void* dst[4] = {ctx->desc.p, ctx->items.p, ctx->item_start.p, ctx->code_off.p};
    const size_t total = sz[0] + sz[1] + sz[2] + sz[3] + 64;
    if (ctx->pinned_bytes < total) {
      HIP_TRY(hipStreamSynchronize(s));
      if (ctx->pinned) HIP_TRY(hipHostFree(ctx->pinned));
      ctx->pinned = nullptr;
      ctx->pinned_bytes = 0;
      HIP_TRY(hipHostMalloc(&ctx->pinned, total, hipHostMallocDefault));
      ctx->pinned_bytes = total;
    }
    HIP_TRY(hipStreamSynchronize(s));  // the staging buffer may still feed the previous call's copies
    size_t o = 0;
    for (int i = 0; i < 4; ++i) {
      std::memcpy(static_cast<uint8_t*>(ctx->pinned) + o, src[i], sz[i]);
      HIP_TRY(hipMemcpyAsync(dst[i], static_cast<uint8_t*>(ctx->pinned) + o, sz[i], hipMemcpyHostToDevice, s));
      o += (sz[i] + 15) & ~size_t(15);
    }
    ctx->plan_valid = true;
    if (std::getenv("DLS_TIMING"))
      std::fprintf(stderr, "[dls] blocks + upload %.3f ms (%zu blocks, %zu items)\n",
                   std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - th0).count(),
                   ctx->plan.blocks.size(), ctx->plan.items.size());
  }
  ctx->prob = p;
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size());
  const int64_t ni = int64_t(pl.items.size());
  const int wp = p.wpad();
  if (p.flags & DLS_GLOBAL) {
    const Dims gdims{p.nx, p.ny, p.nz, p.nt};
    if (dls_status st = global_encode(ctx, d_field, p, gdims, s)) return st;
    return finish_encode(ctx);
  }

  HIP_TRY(ctx->gram.ensure(size_t(ni) * wp * wp * sizeof(double)));
  HIP_TRY(ctx->rank.ensure(size_t(nb)));
  HIP_TRY(ctx->lam.ensure(size_t(nb) * wp * sizeof(double)));
  HIP_TRY(ctx->basis.ensure(size_t(nb) * wp * wp * sizeof(double)));
  HIP_TRY(ctx->qv_size.ensure(size_t(nb) * sizeof(int64_t)));
  HIP_TRY(ctx->qa_size.ensure(size_t(nb) * sizeof(int64_t)));
  HIP_TRY(ctx->qv_off.ensure(size_t(nb) * sizeof(int64_t)));
  HIP_TRY(ctx->qa_off.ensure(size_t(nb) * sizeof(int64_t)));
  HIP_TRY(ctx->scan_tmp.ensure(size_t(4 * (nb / 1024 + 4)) * sizeof(int64_t)));
  HIP_TRY(ctx->codes.ensure(size_t(pl.codes_bytes)));
  HIP_TRY(ctx->counters.ensure(kCounterBytes));
  HIP_TRY(ctx->cls_lists.ensure(size_t(ni) * kEncodeClasses * sizeof(int32_t)));
  if (ctx->esc_cap == 0) {
    ctx->esc_cap = std::max<uint64_t>(uint64_t(1) << 20, uint64_t(p.values() / 256));
    HIP_TRY(ctx->esc_key.ensure(ctx->esc_cap * 8));
    HIP_TRY(ctx->esc_val.ensure(ctx->esc_cap * 8));
  }
  std::vector<VarConst> vc(p.nvars);
  for (int v = 0; v < p.nvars; ++v) vc[v] = var_const(p.eps[v]);
  HIP_TRY(ctx->vconst.ensure(vc.size() * sizeof(VarConst)));
  HIP_TRY(ctx->eps_v.ensure(p.eps.size() * sizeof(double)));
  HIP_TRY(hipMemcpyAsync(ctx->vconst.p, vc.data(), vc.size() * sizeof(VarConst), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(ctx->eps_v.p, p.eps.data(), p.eps.size() * sizeof(double), hipMemcpyHostToDevice, s));
  HIP_TRY(launch_zero(ctx->counters.p, kCounterBytes, s));

  const Dims dims{p.nx, p.ny, p.nz, p.nt};
  unsigned long long* cnt = ctx->counters.as<unsigned long long>();
  if (p.flags & DLS_L2) {
    if (dls_status st = l2_encode(ctx, d_field, p, dims, s)) return st;
    return finish_encode(ctx);
  }
  HIP_TRY(hipEventRecord(ctx->ev0, s));
  // batched: slices of at most kSmallSlice points share workgroups (the split
  // depends on the plan only and is uploaded once per plan)
  const bool batched = (p.flags & DLS_PERSISTENT) != 0;
  if (batched && !ctx->split_valid) {
    std::vector<int32_t> lists[2];
    for (int64_t i = 0; i < ni; ++i) lists[pl.items[i].np <= kSmallSlice ? 1 : 0].push_back(int32_t(i));
    ctx->split_nlarge = int64_t(lists[0].size());
    ctx->split_nsmall = int64_t(lists[1].size());
    HIP_TRY(ctx->split_lists.ensure(size_t(ni) * sizeof(int32_t)));
    HIP_TRY(hipStreamSynchronize(s));  // the pinned staging buffer is reused below
    if (ctx->pinned_bytes < size_t(ni) * sizeof(int32_t)) {
      if (ctx->pinned) HIP_TRY(hipHostFree(ctx->pinned));
      ctx->pinned = nullptr;
      ctx->pinned_bytes = 0;
      HIP_TRY(hipHostMalloc(&ctx->pinned, size_t(ni) * sizeof(int32_t), hipHostMallocDefault));
      ctx->pinned_bytes = size_t(ni) * sizeof(int32_t);
    }
    int32_t* st = static_cast<int32_t*>(ctx->pinned);
    std::copy(lists[0].begin(), lists[0].end(), st);
    std::copy(lists[1].begin(), lists[1].end(), st + lists[0].size());
    HIP_TRY(hipMemcpyAsync(ctx->split_lists.p, st, size_t(ni) * sizeof(int32_t), hipMemcpyHostToDevice, s));
    ctx->split_valid = true;
  }
  const GramSplit split{ctx->split_lists.as<int32_t>(), ctx->split_nlarge,
                        ctx->split_lists.as<int32_t>() + ctx->split_nlarge, ctx->split_nsmall};
  ctx->keep_coef = keep_coef != 0;
  ctx->nfast_accept = ctx->ndeferred = 0;
  ctx->launch_mode = 0;
  // batched plans of large FP32 blocks (W <= 16): the fused single pass
  if (batched && p.dtype == DLS_F32 && wp == 16 && ctx->plan_min_points >= kFusedMinPoints) {
    bool done = false;
    if (dls_status st = fused_encode(ctx, d_field, p, dims, s, &done)) return st;
    if (done) return finish_encode(ctx);
    ctx->nfast_accept = ctx->ndeferred = 0;  // this call is encoded again two-pass
    ctx->fused_timed = ctx->jacobi_timed = false;
    HIP_TRY(hipEventRecord(ctx->ev0, s));
  }
  const bool learned = (p.flags & DLS_LEARNED) != 0;
  const bool warm_any = ctx->plan_warm_blocks > 0;
  unsigned int* overflow = reinterpret_cast<unsigned int*>(reinterpret_cast<uint8_t*>(cnt) + kOverflowAt);
  int64_t* totals = reinterpret_cast<int64_t*>(reinterpret_cast<uint8_t*>(cnt) + kTotalsAt);
  const GramSplit* gsplit = batched ? &split : nullptr;
  // the device-driven launch saves the host round trip (~0.1-0.2 ms) but its
  // looping workgroups encode large lists more slowly than one workgroup per
  // item; measured on the synthetic workloads the crossover lies between
  // ~10^4 and ~2 x 10^5 items, so larger plans keep the host-driven launch
  const bool dd = (p.flags & DLS_PERSISTENT) && ni <= ctx->dd_max_items;
  ctx->dd_replayed = false;
  if (!dd) {
    if (dls_status st = enqueue_front(ctx, d_field, p, dims, gsplit, s, true)) return st;
  } else {
    // device-driven encode into the buffers as they are; one readback at the end
    HIP_TRY(ctx->qv.ensure(16));
    HIP_TRY(ctx->qa.ensure(16));
    if (ctx->keep_coef) HIP_TRY(ctx->coef.ensure(ctx->qa.n));
    uint64_t key[kDdKey];
    dd_key(ctx, d_field, p, key);
    if (ctx->use_graphs && ctx->dd_graph != nullptr && std::equal(key, key + kDdKey, ctx->dd_key)) {
      // replay of the captured sequence; its stages are not separated (the
      // whole replay counts as the encode stage)
      for (int k = 0; k < 4; ++k) HIP_TRY(hipEventRecord(ctx->evs[k], s));
      HIP_TRY(hipGraphLaunch(ctx->dd_graph, s));
      ctx->dd_replayed = true;
    } else {
      if (dls_status st = enqueue_front(ctx, d_field, p, dims, gsplit, s, true)) return st;
      if (dls_status st = enqueue_dd_encode(ctx, d_field, p, dims, s, true)) return st;
    }
    HIP_TRY(hipEventRecord(ctx->ev1, s));
    HIP_TRY(ctx->host_counters());
    HIP_TRY(hipMemcpyAsync(ctx->hcnt, cnt, kCounterBytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint8_t* hbuf = ctx->hcnt;
    unsigned long long hc[4];
    unsigned int hov;
    int64_t ht[2];
    std::memcpy(hc, hbuf, sizeof(hc));
    std::memcpy(&hov, hbuf + kOverflowAt, 4);
    std::memcpy(ht, hbuf + kTotalsAt, sizeof(ht));
    ctx->qv_bytes = ht[0];
    ctx->qa_bytes = ht[1];
    ctx->nesc = ctx->nesc_slots = int64_t(hc[0]);
    ctx->nraw = int64_t(hc[1]);
    ctx->nwarm_accept = learned ? int64_t(hc[2]) : 0;
    ctx->nwarm_reject = learned ? (warm_any ? int64_t(hc[3]) : nb) : 0;
    if (hov == 0 && hc[0] <= ctx->esc_cap) {
      ctx->launch_mode = 1;
      if (ctx->use_graphs && !ctx->dd_replayed) dd_capture(ctx, d_field, p, dims, gsplit);
      return finish_encode(ctx);
    }
    // did not fit: grow with headroom for later calls, then the host-driven
    // encode below rewrites every output
    HIP_TRY(ctx->qv.grow(size_t(ht[0] + ht[0] / 4 + 16)));
    HIP_TRY(ctx->qa.grow(size_t(ht[1] + ht[1] / 4 + 16)));
    if (ctx->keep_coef) HIP_TRY(ctx->coef.grow(ctx->qa.n));
    if (hc[0] > ctx->esc_cap) {
      ctx->esc_cap = hc[0] + (hc[0] >> 3) + 1024;
      HIP_TRY(ctx->esc_key.ensure(ctx->esc_cap * 8));
      HIP_TRY(ctx->esc_val.ensure(ctx->esc_cap * 8));
    }
    HIP_TRY(launch_zero(cnt, sizeof(unsigned long long), s));
  }
  // class counts and payload totals in one readback into pinned memory
  HIP_TRY(launch_totals(ctx->qv_off.as<int64_t>(), ctx->qv_size.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                        ctx->qa_size.as<int64_t>(), nb, totals, s));
  HIP_TRY(ctx->host_counters());
  HIP_TRY(hipMemcpyAsync(ctx->hcnt, cnt, kCounterBytes, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  unsigned int hcls[kEncodeClasses];
  int64_t htot[2];
  std::memcpy(hcls, ctx->hcnt + 4 * sizeof(unsigned long long), sizeof(hcls));
  std::memcpy(htot, ctx->hcnt + kTotalsAt, sizeof(htot));
  ctx->qv_bytes = htot[0];
  ctx->qa_bytes = htot[1];
  HIP_TRY(ctx->qv.ensure(size_t(ctx->qv_bytes)));
  HIP_TRY(ctx->qa.ensure(size_t(ctx->qa_bytes)));
  if (ctx->keep_coef) HIP_TRY(ctx->coef.ensure(size_t(ctx->qa_bytes)));

  for (int attempt = 0; attempt < 2; ++attempt) {
    EscOut esc{cnt, ctx->esc_key.as<uint64_t>(), ctx->esc_val.as<uint64_t>(), ctx->esc_cap};
    HIP_TRY(hipEventRecord(ctx->evs[3], s));
    for (int c = 0; c < kEncodeClasses; ++c)
      HIP_TRY(launch_encode(wp, p.dtype, c, d_field, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(),
                            ctx->cls_lists.as<int32_t>() + int64_t(c) * ni,
                            EncodeWork{nullptr, int64_t(hcls[c]), int64_t(ctx->qv.n), int64_t(ctx->qa.n), overflow},
                            ctx->rank.as<uint8_t>(),
                            ctx->basis.as<double>(), ctx->qv_off.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                            ctx->code_off.as<int64_t>(), ctx->vconst.as<VarConst>(), ctx->qv.as<uint8_t>(),
                            ctx->qa.as<uint8_t>(), ctx->codes.as<uint8_t>(),
                            ctx->keep_coef ? ctx->coef.as<float>() : nullptr, esc, s));
    HIP_TRY(hipEventRecord(ctx->ev1, s));
    unsigned long long hc[4];
    HIP_TRY(hipMemcpyAsync(ctx->hcnt, cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(hc, ctx->hcnt, sizeof(hc));
    ctx->nesc = ctx->nesc_slots = int64_t(hc[0]);
    ctx->nraw = int64_t(hc[1]);
    ctx->nwarm_accept = learned ? int64_t(hc[2]) : 0;
    ctx->nwarm_reject = learned ? (warm_any ? int64_t(hc[3]) : nb) : 0;
    if (hc[0] <= ctx->esc_cap) break;
    // more escapes than room: grow and run the encode kernel again (it rewrites
    // every output, so the result is identical apart from the escape list)
    ctx->esc_cap = hc[0] + (hc[0] >> 3) + 1024;
    HIP_TRY(ctx->esc_key.ensure(ctx->esc_cap * 8));
    HIP_TRY(ctx->esc_val.ensure(ctx->esc_cap * 8));
    HIP_TRY(launch_zero(cnt, sizeof(unsigned long long), s));
  }
  return finish_encode(ctx);
}

dls_status dls_model_create(int device, dls_model** out) {
  if (out == nullptr) return fail(DLS_EINVAL, "out is NULL");
  *out = nullptr;
  int n = 0;
  HIP_TRY(hipGetDeviceCount(&n));
  if (device < 0 || device >= n) return fail(DLS_EINVAL, "no such device");
  HIP_TRY(hipSetDevice(device));
  std::unique_ptr<dls_model> m(new (std::nothrow) dls_model());
  if (!m) return fail(DLS_ENOMEM, "model allocation");
  m->device = device;
  HIP_TRY(m->params.ensure(kNParam * 4));
  HIP_TRY(m->grad.ensure(kNParam * 4));
  HIP_TRY(m->m.ensure(kNParam * 4));
  HIP_TRY(m->v.ensure(kNParam * 4));
  HIP_TRY(m->norm.ensure(32 * 4));
  HIP_TRY(hipMemset(m->params.p, 0, kNParam * 4));
  HIP_TRY(hipMemset(m->grad.p, 0, kNParam * 4));
  HIP_TRY(hipMemset(m->m.p, 0, kNParam * 4));
  HIP_TRY(hipMemset(m->v.p, 0, kNParam * 4));
  std::vector<float> norm(32, 0.f);
  for (int i = 16; i < 32; ++i) norm[i] = 1.f;
  HIP_TRY(hipMemcpy(m->norm.p, norm.data(), 32 * 4, hipMemcpyHostToDevice));
  *out = m.release();
  return DLS_OK;
}

void dls_model_destroy(dls_model* m) {
  if (m == nullptr) return;
  (void)hipSetDevice(m->device);
  delete m;
}

dls_status dls_model_set(dls_model* m, const float* params, const float* norm) {
  if (m == nullptr || params == nullptr) return fail(DLS_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(m->device));
  if (norm != nullptr)
    for (int i = 16; i < 32; ++i)
      if (!(norm[i] > 0.f)) return fail(DLS_EINVAL, "normalisation scales must be > 0");
  HIP_TRY(hipMemcpy(m->params.p, params, kNParam * 4, hipMemcpyHostToDevice));
  m->packed_valid = false;
  ++m->version;
  if (norm != nullptr) HIP_TRY(hipMemcpy(m->norm.p, norm, 32 * 4, hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(m->m.p, 0, kNParam * 4));
  HIP_TRY(hipMemset(m->v.p, 0, kNParam * 4));
  m->step = 0;
  return DLS_OK;
}

dls_status dls_model_get(const dls_model* m, float* params, float* norm) {
  if (m == nullptr) return fail(DLS_EINVAL, "NULL model");
  HIP_TRY(hipSetDevice(m->device));
  if (params != nullptr) HIP_TRY(hipMemcpy(params, m->params.p, kNParam * 4, hipMemcpyDeviceToHost));
  if (norm != nullptr) HIP_TRY(hipMemcpy(norm, m->norm.p, 32 * 4, hipMemcpyDeviceToHost));
  return DLS_OK;
}

dls_status dls_model_forward(dls_model* m, const float* d_feat, int64_t n, int bf16, float* d_out, void* stream) {
  if (m == nullptr || d_feat == nullptr || d_out == nullptr || n < 1 || bf16 < 0 || bf16 > 2)
    return fail(DLS_EINVAL, "bad argument");
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (bf16 == 1) {
    if (dls_status st = model_infer(m, d_feat, n, d_out, s)) return st;
  } else {
    if (dls_status st = model_workspace(m, n)) return st;
    if (dls_status st = model_forward(m, d_feat, n, bf16 != 0, d_out, s)) return st;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return DLS_OK;
}

dls_status dls_model_grad(dls_model* m, const float* d_feat, const int32_t* d_rank, const float* d_basis,
                          const int32_t* d_wb, int64_t n, int bf16, float* d_grad, float* loss_out, void* stream) {
  if (m == nullptr || d_feat == nullptr || d_rank == nullptr || d_basis == nullptr || d_wb == nullptr ||
      d_grad == nullptr || n < 1)
    return fail(DLS_EINVAL, "bad argument");
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dls_status st = model_backprop(m, d_feat, d_rank, d_basis, d_wb, n, bf16 != 0, loss_out, s)) return st;
  HIP_TRY(hipMemcpyAsync(d_grad, m->grad.p, kNParam * 4, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DLS_OK;
}

dls_status dls_model_train_step(dls_model* m, const float* d_feat, const int32_t* d_rank, const float* d_basis,
                                const int32_t* d_wb, int64_t n, float lr, int bf16, float* loss_out,
                                void* stream) {
  if (m == nullptr || d_feat == nullptr || d_rank == nullptr || d_basis == nullptr || d_wb == nullptr || n < 1 ||
      !(lr > 0.f))
    return fail(DLS_EINVAL, "bad argument");
  HIP_TRY(hipSetDevice(m->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (dls_status st = model_backprop(m, d_feat, d_rank, d_basis, d_wb, n, bf16 != 0, loss_out, s)) return st;
  m->step += 1;
  const float c1 = float(1.0 - std::pow(0.9, double(m->step)));
  const float c2 = float(1.0 - std::pow(0.999, double(m->step)));
  m->packed_valid = false;
  ++m->version;
  HIP_TRY(launch_adam(m->params.as<float>(), m->grad.as<float>(), m->m.as<float>(), m->v.as<float>(), kNParam, lr, c1,
                      c2, s));
  if (loss_out == nullptr) HIP_TRY(hipStreamSynchronize(s));
  return DLS_OK;
}

dls_status dls_decode(dls_ctx* ctx, void* d_out, size_t out_bytes, void* stream) {
  if (ctx == nullptr || d_out == nullptr) return fail(DLS_EINVAL, "NULL argument");
  if (!ctx->have_result) return fail(DLS_EINVAL, "no encode result in this context");
  const Problem& p = ctx->prob;
  if (out_bytes < size_t(p.values()) * size_t(p.esize()))
    return fail(DLS_EINVAL, "output buffer smaller than the encoded field");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Dims dims{p.nx, p.ny, p.nz, p.nt};
  if (p.flags & DLS_L2) {
    HIP_TRY(launch_l2_decode(p.wpad(), p.dtype, d_out, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(),
                             int64_t(ctx->plan.items.size()), ctx->l2rank.as<uint8_t>(), ctx->l2step.as<double>(),
                             ctx->qv_off.as<int64_t>(), ctx->qa_off.as<int64_t>(), ctx->qv.as<uint8_t>(),
                             ctx->qa.as<uint8_t>(), s));
    return DLS_OK;
  }
  if (p.flags & DLS_GLOBAL) {
    HIP_TRY(launch_gb_decode(p.dtype, d_out, dims, ctx->desc.as<BlockDesc>(), int64_t(ctx->plan.blocks.size()),
                             p.nvars, ctx->gb_phi.as<double>(), p.px, p.py, ctx->gb_M, ctx->gb_count.as<int32_t>(),
                             ctx->gb_kexp.as<int32_t>(), ctx->gb_idx_off.as<int64_t>(), ctx->gb_raw_off.as<int64_t>(),
                             ctx->gb_idx.as<uint16_t>(), ctx->gb_q.as<int32_t>(), ctx->gb_raw.as<uint8_t>(), s));
    return DLS_OK;
  }
  // one launch per rank class, over the encode's class lists (their counts
  // are in the host copy of the counter block the encode read back last)
  const int64_t ni = int64_t(ctx->plan.items.size());
  unsigned int hcls[kEncodeClasses];
  std::memcpy(hcls, ctx->hcnt + 4 * sizeof(unsigned long long), sizeof(hcls));
  for (int c = 0; c < kEncodeClasses; ++c)
    HIP_TRY(launch_decode_class(p.wpad(), p.dtype, c % kRankClasses, c >= kRankClasses,
                                ctx->cls_lists.as<int32_t>() + int64_t(c) * ni,
                                int64_t(hcls[c]), d_out, dims, ctx->desc.as<BlockDesc>(), ctx->items.as<Item>(),
                                ctx->rank.as<uint8_t>(), ctx->qv_off.as<int64_t>(), ctx->qa_off.as<int64_t>(),
                                ctx->code_off.as<int64_t>(), ctx->vconst.as<VarConst>(), ctx->qv.as<uint8_t>(),
                                ctx->qa.as<uint8_t>(), ctx->codes.as<uint8_t>(), s));
  HIP_TRY(launch_scatter_keys(p.dtype, d_out, dims, ctx->desc.as<BlockDesc>(), ctx->esc_key.as<uint64_t>(),
                              ctx->esc_val.as<uint64_t>(), ctx->nesc_slots, s));
  return DLS_OK;
}

dls_status dls_features(dls_ctx* ctx, const void* d_field, size_t field_bytes, float* d_out, size_t out_bytes,
                        void* stream) {
  if (ctx == nullptr || d_field == nullptr || d_out == nullptr) return fail(DLS_EINVAL, "NULL argument");
  if (!ctx->have_result) return fail(DLS_EINVAL, "no encode result in this context");
  const Problem& p = ctx->prob;
  if (field_bytes < size_t(p.values()) * size_t(p.esize()))
    return fail(DLS_EINVAL, "field buffer smaller than the encoded field");
  if (out_bytes < ctx->plan.blocks.size() * size_t(kNF) * sizeof(float))
    return fail(DLS_EINVAL, "output buffer smaller than nblocks x 80 floats");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (p.window > 16) return fail(DLS_EINVAL, "features need window <= 16");
  const Dims dims{p.nx, p.ny, p.nz, p.nt};
  FeatureLists fl;
  if (dls_status st = feature_lists(ctx, fl)) return st;
  HIP_TRY(launch_features(p.dtype, d_field, dims, ctx->desc.as<BlockDesc>(), fl, ctx->eps_v.as<double>(), d_out, s));
  HIP_TRY(hipStreamSynchronize(s));
  return DLS_OK;
}

dls_status dls_ctx_set_model(dls_ctx* ctx, dls_model* m, int iters, int rank_margin) {
  if (ctx == nullptr || iters < 0 || iters > 64 || rank_margin < 0 || rank_margin > 16)
    return fail(DLS_EINVAL, "bad argument");
  ctx->model = m;
  ctx->warm_iters = iters;
  ctx->warm_margin = rank_margin;
  return DLS_OK;
}

dls_status dls_range(const void* d_field, int32_t nvars, int64_t values_per_var, int32_t dtype,
                     void* stream, double* min_out, double* max_out) {
  if (d_field == nullptr || min_out == nullptr || max_out == nullptr) return fail(DLS_EINVAL, "NULL argument");
  if (nvars < 1 || values_per_var < 1) return fail(DLS_EINVAL, "empty field");
  if (dtype != DLS_F32 && dtype != DLS_F64) return fail(DLS_EINVAL, "bad dtype");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nparts = int(std::min<int64_t>(kRangeParts, (values_per_var + 255) / 256));
  DevBuf part, out;
  HIP_TRY(part.ensure(size_t(nvars) * nparts * 2 * sizeof(double)));
  HIP_TRY(out.ensure(size_t(nvars) * 2 * sizeof(double)));
  HIP_TRY(launch_range(dtype, d_field, nvars, values_per_var, part.as<double>(), nparts, out.as<double>(), s));
  std::vector<double> h(2 * size_t(nvars));
  HIP_TRY(hipMemcpyAsync(h.data(), out.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int v = 0; v < nvars; ++v) {
    min_out[v] = h[2 * v];
    max_out[v] = h[2 * v + 1];
  }
  return DLS_OK;
}

dls_status dls_range_noalloc(const void* d_field, int32_t nvars, int64_t values_per_var, int32_t dtype,
                             void* stream, double* min_out, double* max_out) {
  if (d_field == nullptr || min_out == nullptr || max_out == nullptr) return fail(DLS_EINVAL, "NULL argument");
  if (nvars < 1 || values_per_var < 1) return fail(DLS_EINVAL, "empty field");
  if (nvars > kRangeNoAllocVars) return fail(DLS_EINVAL, "dls_range_noalloc takes at most 64 variables");
  if (dtype != DLS_F32 && dtype != DLS_F64) return fail(DLS_EINVAL, "bad dtype");
  hipStream_t s = static_cast<hipStream_t>(stream);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  double* sp = nullptr;  // this device's copy of the library's fixed range scratch
  HIP_TRY(range_scratch(dev, &sp));
  HIP_TRY(launch_range_noalloc(sp, dtype, d_field, nvars, values_per_var, s));
  double h[2 * kRangeNoAllocVars];
  HIP_TRY(hipMemcpyAsync(h, sp + int64_t(nvars) * 2 * kRangeParts, size_t(2 * nvars) * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int v = 0; v < nvars; ++v) {
    min_out[v] = h[2 * v];
    max_out[v] = h[2 * v + 1];
  }
  return DLS_OK;
}

dls_status dls_encode_info_get(const dls_ctx* ctx, dls_encode_info* info) {
  if (ctx == nullptr || info == nullptr) return fail(DLS_EINVAL, "NULL argument");
  if (!ctx->have_result) return fail(DLS_EINVAL, "no encode result in this context");
  info->nblocks = int64_t(ctx->plan.blocks.size());
  info->nescapes = ctx->nesc;
  info->nraw = ctx->nraw;
  info->wpad = ctx->prob.wpad();
  info->d_rank = ctx->rank.as<uint8_t>();
  info->d_lam = ctx->lam.as<double>();
  info->d_basis = ctx->basis.as<double>();
  info->d_desc = ctx->desc.as<int32_t>();
  info->qa_bytes = ctx->qa_bytes;
  info->codes_bytes = ctx->plan.codes_bytes;
  info->d_qa = ctx->qa.as<uint8_t>();
  info->d_codes = ctx->codes.as<uint8_t>();
  info->d_qa_off = ctx->qa_off.as<int64_t>();
  info->d_code_off = ctx->code_off.as<int64_t>();
  info->d_coef = ctx->keep_coef ? ctx->coef.as<float>() : nullptr;
  info->nwarm_accept = ctx->nwarm_accept;
  info->nwarm_reject = ctx->nwarm_reject;
  info->nfast_accept = ctx->nfast_accept;
  info->ndeferred = ctx->ndeferred;
  info->launch_mode = ctx->launch_mode;
  info->npredicted_deferred = ctx->npredicted;
  info->npruned = ctx->npruned;
  info->fused_declined = ctx->fused_declined ? 1 : 0;
  info->l2_passes = (ctx->prob.flags & DLS_L2) ? ctx->l2_passes : 0;
  info->jacobi_sweeps = ctx->jacobi_sweeps;
  info->jacobi_unconverged = ctx->jacobi_unconverged;
  info->jacobi_ms = ctx->jacobi_ms;
  info->fused_ms = ctx->fused_ms;
  info->gpu_ms = ctx->gpu_ms;
  for (int i = 0; i < 5; ++i) info->stage_ms[i] = ctx->stage_ms[i];
  return DLS_OK;
}

dls_status dls_finalize(dls_ctx* ctx, uint8_t** out, size_t* out_bytes) {
  if (ctx == nullptr || out == nullptr || out_bytes == nullptr) return fail(DLS_EINVAL, "NULL argument");
  if (!ctx->have_result) return fail(DLS_EINVAL, "no encode result in this context");
  *out = nullptr;
  *out_bytes = 0;
  HIP_TRY(hipSetDevice(ctx->device));
  if (ctx->prob.flags & DLS_L2) return l2_finalize(ctx, out, out_bytes);
  if (ctx->prob.flags & DLS_GLOBAL) return global_finalize(ctx, out, out_bytes);
  const Problem& p = ctx->prob;
  const Plan& pl = ctx->plan;
  const int64_t nb = int64_t(pl.blocks.size());
  std::vector<uint8_t> rank(nb), qv(ctx->qv_bytes), qa(ctx->qa_bytes), codes(pl.codes_bytes);
  std::vector<int64_t> qv_off(nb), qa_off(nb);
  std::vector<uint64_t> ekey(ctx->nesc_slots), eval(ctx->nesc_slots);
  HIP_TRY(hipMemcpy(rank.data(), ctx->rank.p, nb, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(qv_off.data(), ctx->qv_off.p, nb * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(qa_off.data(), ctx->qa_off.p, nb * 8, hipMemcpyDeviceToHost));
  if (ctx->qv_bytes) HIP_TRY(hipMemcpy(qv.data(), ctx->qv.p, ctx->qv_bytes, hipMemcpyDeviceToHost));
  if (ctx->qa_bytes) HIP_TRY(hipMemcpy(qa.data(), ctx->qa.p, ctx->qa_bytes, hipMemcpyDeviceToHost));
  if (pl.codes_bytes) HIP_TRY(hipMemcpy(codes.data(), ctx->codes.p, pl.codes_bytes, hipMemcpyDeviceToHost));
  if (ctx->nesc_slots) {
    HIP_TRY(hipMemcpy(ekey.data(), ctx->esc_key.p, ctx->nesc_slots * 8, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(eval.data(), ctx->esc_val.p, ctx->nesc_slots * 8, hipMemcpyDeviceToHost));
  }
  // escapes in block, then (t, p) order; entries the single pass dropped
  // (key ~0) sort last and are left out
  std::vector<int64_t> order(ctx->nesc_slots);
  for (int64_t i = 0; i < ctx->nesc_slots; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return ekey[a] < ekey[b]; });
  order.resize(ctx->nesc);
  std::vector<int64_t> esc_start(nb + 1, 0);
  for (int64_t i = 0; i < ctx->nesc; ++i) esc_start[(ekey[order[i]] >> 32) + 1]++;
  for (int64_t b = 0; b < nb; ++b) esc_start[b + 1] += esc_start[b];

  const int64_t nbatch = (nb + kBatchBlocks - 1) / kBatchBlocks;
  const int es = p.esize();
  std::vector<std::vector<uint8_t>> zs(nbatch);
  std::vector<uint64_t> usz(nbatch);
  std::atomic<bool> zfail{false};
  parallel_for(nbatch, [&](int64_t bi) {
    const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks);
    std::vector<uint8_t> raw;
    size_t need = (b1 - b0) * 5;
    for (int64_t b = b0; b < b1; ++b) {
      const BlockDesc& d = pl.blocks[b];
      need += size_t(4) * rank[b] * (d.w() + d.m) + size_t(2) * d.w() * d.m + size_t(es) * (esc_start[b + 1] - esc_start[b]);
    }
    raw.reserve(need);
    raw.insert(raw.end(), rank.begin() + b0, rank.begin() + b1);
    for (int64_t b = b0; b < b1; ++b) {
      uint32_t c = uint32_t(esc_start[b + 1] - esc_start[b]);
      uint8_t tmp[4];
      std::memcpy(tmp, &c, 4);
      raw.insert(raw.end(), tmp, tmp + 4);
    }
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t n = int64_t(pl.blocks[b].w()) * rank[b], pad = pad16(n);
      for (int j = 0; j < 4; ++j) {
        const uint8_t* src = qv.data() + qv_off[b] + j * pad;
        raw.insert(raw.end(), src, src + n);
      }
    }
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t n = int64_t(pl.blocks[b].m) * rank[b], pad = pad16(n);
      for (int j = 0; j < 4; ++j) {
        const uint8_t* src = qa.data() + qa_off[b] + j * pad;
        raw.insert(raw.end(), src, src + n);
      }
    }
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t n = int64_t(pl.blocks[b].w()) * pl.blocks[b].m;
      const uint8_t* src = codes.data() + pl.code_off[b];
      raw.insert(raw.end(), src, src + n);
    }
    for (int64_t i = esc_start[b0]; i < esc_start[b1]; ++i) {
      uint8_t tmp[8];
      std::memcpy(tmp, &eval[order[i]], 8);
      raw.insert(raw.end(), tmp, tmp + es);
    }
    uLongf zn = compressBound(uLong(raw.size()));
    std::vector<uint8_t> z(zn);
    if (compress2(z.data(), &zn, raw.data(), uLong(raw.size()), kZlibLevel) != Z_OK) {
      zfail = true;
      return;
    }
    z.resize(zn);
    zs[bi] = std::move(z);
    usz[bi] = raw.size();
  });
  if (zfail) return fail(DLS_ENOMEM, "zlib compress2 failed");
  std::vector<StreamHeader::Batch> table(nbatch);
  uint64_t off = 0;
  for (int64_t i = 0; i < nbatch; ++i) {
    table[i] = StreamHeader::Batch{off, zs[i].size(), usz[i]};
    off += zs[i].size();
  }
  std::vector<uint8_t> hdr = write_header(p, nb, pl.bits, table);
  const size_t total = hdr.size() + off;
  uint8_t* buf = static_cast<uint8_t*>(std::malloc(total ? total : 1));
  if (buf == nullptr) return fail(DLS_ENOMEM, "output allocation");
  std::memcpy(buf, hdr.data(), hdr.size());
  size_t pos = hdr.size();
  for (auto& z : zs) {
    std::memcpy(buf + pos, z.data(), z.size());
    pos += z.size();
  }
  *out = buf;
  *out_bytes = total;
  return DLS_OK;
}

dls_status dls_compress(const void* d_field, const dls_params* p, void* stream, uint8_t** out,
                        size_t* out_bytes) {
  if (out == nullptr || out_bytes == nullptr) return fail(DLS_EINVAL, "NULL output argument");
  if (d_field == nullptr) return fail(DLS_EINVAL, "field is NULL");
  Problem chk;
  if (dls_status s = validate(p, chk)) return s;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  dls_ctx* ctx = nullptr;
  if (dls_status s = dls_ctx_create(dev, &ctx)) return s;
  dls_status s = DLS_OK;
  if (p->model != nullptr) s = dls_ctx_set_model(ctx, p->model, p->warm_iters > 0 ? p->warm_iters : 2, p->rank_margin);
  if (s == DLS_OK) s = dls_encode(ctx, d_field, p, stream, 0);
  if (s == DLS_OK) s = dls_finalize(ctx, out, out_bytes);
  dls_ctx_destroy(ctx);
  return s;
}

dls_status dls_query(const uint8_t* in, size_t in_bytes, dls_params* p_out, double* eps_out,
                     int32_t eps_cap, int64_t* nblocks) {
  if (p_out == nullptr) return fail(DLS_EINVAL, "p_out is NULL");
  StreamHeader h;
  std::string err = parse_header(in, in_bytes, h);
  if (!err.empty()) return fail(DLS_ECORRUPT, err);
  const Problem& p = h.prob;
  std::memset(p_out, 0, sizeof(*p_out));
  p_out->struct_size = sizeof(dls_params);
  p_out->nvars = p.nvars;
  p_out->nx = p.nx; p_out->ny = p.ny; p_out->nz = p.nz; p_out->nt = p.nt;
  p_out->dtype = p.dtype;
  p_out->px = p.px; p_out->py = p.py; p_out->pz = p.pz; p_out->pmin = p.pmin;
  p_out->window = p.window;
  p_out->r_max = p.r_max;
  p_out->precision = 0;
  p_out->flags = p.flags;
  p_out->abs_eps = nullptr;
  p_out->basis = (p.flags & DLS_GLOBAL) ? int32_t(h.extra) : 0;
  if (eps_out != nullptr)
    for (int v = 0; v < std::min<int>(p.nvars, std::max(0, eps_cap)); ++v) eps_out[v] = p.eps[v];
  if (nblocks != nullptr) *nblocks = h.nblocks;
  return DLS_OK;
}

}  // extern "C"

namespace {

// Host view of one inflated batch, split into its sections.
struct BatchView {
  std::vector<uint8_t> raw;
  size_t ranks = 0, esc = 0, qv = 0, qa = 0, codes = 0, vals = 0;
};

// Inflate batch bi and locate its sections; "" on success.
std::string inflate_batch(const uint8_t* in, const StreamHeader& h, const Plan& pl, int64_t bi, BatchView& bv) {
  const auto& e = h.batches[bi];
  if (e.usize > (uint64_t(1) << 40)) return "batch too large";
  bv.raw.resize(e.usize);
  uLongf n = uLongf(e.usize);
  if (uncompress(bv.raw.data(), &n, in + h.header_bytes + e.off, uLong(e.csize)) != Z_OK || n != e.usize)
    return "zlib stream of a batch is corrupt";
  const int64_t nb = int64_t(pl.blocks.size());
  const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks);
  const int64_t cnt = b1 - b0;
  size_t pos = 0;
  auto need = [&](size_t k) { return pos + k <= bv.raw.size(); };
  if (!need(5 * cnt)) return "batch payload truncated";
  bv.ranks = 0;
  bv.esc = cnt;
  pos = 5 * cnt;
  bv.qv = pos;
  for (int64_t b = b0; b < b1; ++b) {
    const int r = bv.raw[b - b0];
    const BlockDesc& d = pl.blocks[b];
    if (r > std::min({h.prob.r_max, d.w(), d.m})) return "rank out of range";
    pos += size_t(4) * d.w() * r;
  }
  bv.qa = pos;
  for (int64_t b = b0; b < b1; ++b) pos += size_t(4) * pl.blocks[b].m * bv.raw[b - b0];
  bv.codes = pos;
  for (int64_t b = b0; b < b1; ++b) pos += size_t(pl.blocks[b].w()) * pl.blocks[b].m;
  bv.vals = pos;
  int64_t nesc = 0;
  for (int64_t j = 0; j < cnt; ++j) {
    uint32_t c;
    std::memcpy(&c, bv.raw.data() + cnt + 4 * j, 4);
    nesc += c;
  }
  pos += size_t(h.prob.esize()) * size_t(nesc);
  if (pos != bv.raw.size()) return "batch payload size mismatch";
  return "";
}

}  // namespace

extern "C" {

dls_status dls_stats(const uint8_t* in, size_t in_bytes, dls_stream_stats* s) {
  if (s == nullptr) return fail(DLS_EINVAL, "s is NULL");
  StreamHeader h;
  std::string err = parse_header(in, in_bytes, h);
  if (!err.empty()) return fail(DLS_ECORRUPT, err);
  Plan pl;
  err = plan_from_header(h, pl, 1024);
  if (!err.empty()) return fail(DLS_ECORRUPT, err);
  std::memset(s, 0, sizeof(*s));
  s->nblocks = h.nblocks;
  s->nbatches = int64_t(h.batches.size());
  s->stream_bytes = int64_t(in_bytes);
  if (h.prob.flags & DLS_GLOBAL) {
    // coefficient counts per patch-snapshot: rank_hist[min(n, 32)]
    GlobalPayload g;
    err = global_unpack(in, h, pl, g);
    if (!err.empty()) return fail(DLS_ECORRUPT, err);
    for (int32_t c : g.cnt) {
      if (c == kGbRaw) s->nraw++;
      else s->rank_hist[std::min(c, 32)]++;
    }
    for (const auto& e : h.batches) s->payload_bytes += int64_t(e.usize);
    return DLS_OK;
  }
  if (h.prob.flags & DLS_L2) {
    for (int64_t bi = 0; bi < s->nbatches; ++bi) {
      const auto& e = h.batches[bi];
      if (e.usize > (uint64_t(1) << 40)) return fail(DLS_ECORRUPT, "batch too large");
      std::vector<uint8_t> raw(e.usize);
      uLongf n = uLongf(e.usize);
      if (uncompress(raw.data(), &n, in + h.header_bytes + e.off, uLong(e.csize)) != Z_OK || n != e.usize)
        return fail(DLS_ECORRUPT, "zlib stream of a batch is corrupt");
      const int64_t cnt = std::min<int64_t>(kBatchBlocks, h.nblocks - bi * kBatchBlocks);
      if (int64_t(raw.size()) < 9 * cnt) return fail(DLS_ECORRUPT, "batch payload truncated");
      for (int64_t j = 0; j < cnt; ++j) {
        const int r = raw[j];
        if (r == kL2Raw) s->nraw++;
        else if (r <= 32) s->rank_hist[r]++;
        else return fail(DLS_ECORRUPT, "rank out of range");
      }
      s->payload_bytes += int64_t(raw.size());
    }
    return DLS_OK;
  }
  for (int64_t bi = 0; bi < s->nbatches; ++bi) {
    BatchView bv;
    err = inflate_batch(in, h, pl, bi, bv);
    if (!err.empty()) return fail(DLS_ECORRUPT, err);
    const int64_t cnt = int64_t(bv.esc);
    for (int64_t j = 0; j < cnt; ++j) {
      const int r = bv.raw[j];
      s->rank_hist[r]++;
      if (r == 0) s->nraw++;
      uint32_t c;
      std::memcpy(&c, bv.raw.data() + cnt + 4 * j, 4);
      s->nescapes += c;
    }
    s->payload_bytes += int64_t(bv.raw.size());
  }
  return DLS_OK;
}

dls_status dls_decompress(const uint8_t* in, size_t in_bytes, void* d_out, void* stream) {
  if (d_out == nullptr) return fail(DLS_EINVAL, "output is NULL");
  StreamHeader h;
  std::string err = parse_header(in, in_bytes, h);
  if (!err.empty()) return fail(DLS_ECORRUPT, err);
  const Problem& p = h.prob;
  Plan pl;
  err = plan_from_header(h, pl, 1024);
  if (!err.empty()) return fail(DLS_ECORRUPT, err);
  if (p.flags & DLS_L2) return l2_decompress(in, h, pl, d_out, static_cast<hipStream_t>(stream));
  if (p.flags & DLS_GLOBAL) return global_decompress(in, h, pl, d_out, static_cast<hipStream_t>(stream));
  const int64_t nb = h.nblocks, nbatch = int64_t(h.batches.size());
  std::vector<BatchView> views(nbatch);
  std::vector<std::string> errs(nbatch);
  parallel_for(nbatch, [&](int64_t bi) { errs[bi] = inflate_batch(in, h, pl, bi, views[bi]); });
  for (auto& e : errs)
    if (!e.empty()) return fail(DLS_ECORRUPT, e);

  // device layout of the payload (same padding rules as the encoder)
  std::vector<uint8_t> rank(nb);
  std::vector<int64_t> qv_off(nb), qa_off(nb);
  int64_t qv_bytes = 0, qa_bytes = 0;
  for (int64_t b = 0; b < nb; ++b) {
    const BlockDesc& d = pl.blocks[b];
    const int r = views[b / kBatchBlocks].raw[b % kBatchBlocks];
    rank[b] = uint8_t(r);
    qv_off[b] = qv_bytes;
    qa_off[b] = qa_bytes;
    qv_bytes += 4 * pad16(int64_t(d.w()) * r);
    qa_bytes += 4 * pad16(int64_t(d.m) * r);
  }
  std::vector<uint8_t> qv(std::max<int64_t>(qv_bytes, 1)), qa(std::max<int64_t>(qa_bytes, 1)),
      codes(std::max<int64_t>(pl.codes_bytes, 1));
  std::vector<std::vector<int64_t>> eidx(nbatch);
  std::vector<std::vector<uint64_t>> ebits(nbatch);
  const int es = p.esize();
  const Dims dims{p.nx, p.ny, p.nz, p.nt};
  parallel_for(nbatch, [&](int64_t bi) {
    BatchView& bv = views[bi];
    const int64_t b0 = bi * kBatchBlocks, b1 = std::min(nb, b0 + kBatchBlocks);
    const int64_t cnt = b1 - b0;
    size_t pv = bv.qv, pa = bv.qa, pc = bv.codes, pe = bv.vals;
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t n = int64_t(pl.blocks[b].w()) * rank[b], pad = pad16(n);
      for (int j = 0; j < 4; ++j, pv += n) std::memcpy(qv.data() + qv_off[b] + j * pad, bv.raw.data() + pv, n);
    }
    for (int64_t b = b0; b < b1; ++b) {
      const int64_t n = int64_t(pl.blocks[b].m) * rank[b], pad = pad16(n);
      for (int j = 0; j < 4; ++j, pa += n) std::memcpy(qa.data() + qa_off[b] + j * pad, bv.raw.data() + pa, n);
    }
    for (int64_t b = b0; b < b1; ++b) {
      const BlockDesc& d = pl.blocks[b];
      const int64_t n = int64_t(d.w()) * d.m;
      const uint8_t* cd = bv.raw.data() + pc;
      std::memcpy(codes.data() + pl.code_off[b], cd, n);
      uint32_t want;
      std::memcpy(&want, bv.raw.data() + cnt + 4 * (b - b0), 4);
      uint32_t got = 0;
      for (int64_t i = 0; i < n; ++i) {
        if (cd[i] == kEscCode) {
          const int t = int(i / d.m), pt = int(i % d.m);
          const int ii = pt % d.px(), rho = pt / d.px(), jj = rho % d.py(), kk = rho / d.py();
          const int64_t fi = (((int64_t(d.var) * dims.nt + d.t0 + t) * dims.nz + d.z0 + kk) * dims.ny + d.y0 + jj) *
                                 dims.nx + d.x0 + ii;
          uint64_t v = 0;
          if (pe + es <= bv.raw.size()) std::memcpy(&v, bv.raw.data() + pe, es);
          pe += es;
          eidx[bi].push_back(fi);
          ebits[bi].push_back(v);
          ++got;
        }
      }
      if (got != want) {
        errs[bi] = "escape count mismatch";
        return;
      }
      pc += n;
    }
  });
  for (auto& e : errs)
    if (!e.empty()) return fail(DLS_ECORRUPT, e);
  std::vector<int64_t> all_idx;
  std::vector<uint64_t> all_bits;
  for (int64_t bi = 0; bi < nbatch; ++bi) {
    all_idx.insert(all_idx.end(), eidx[bi].begin(), eidx[bi].end());
    all_bits.insert(all_bits.end(), ebits[bi].begin(), ebits[bi].end());
  }
  std::vector<VarConst> vc(p.nvars);
  for (int v = 0; v < p.nvars; ++v) vc[v] = var_const(p.eps[v]);

  hipStream_t s = static_cast<hipStream_t>(stream);
  DevBuf d_desc, d_items, d_rank, d_qvo, d_qao, d_codeo, d_vc, d_qv, d_qa, d_codes, d_eidx, d_ebits;
  HIP_TRY(d_desc.ensure(pl.blocks.size() * sizeof(BlockDesc)));
  HIP_TRY(d_items.ensure(pl.items.size() * sizeof(Item)));
  HIP_TRY(d_rank.ensure(nb));
  HIP_TRY(d_qvo.ensure(nb * 8));
  HIP_TRY(d_qao.ensure(nb * 8));
  HIP_TRY(d_codeo.ensure(nb * 8));
  HIP_TRY(d_vc.ensure(vc.size() * sizeof(VarConst)));
  HIP_TRY(d_qv.ensure(qv.size()));
  HIP_TRY(d_qa.ensure(qa.size()));
  HIP_TRY(d_codes.ensure(codes.size()));
  HIP_TRY(d_eidx.ensure(all_idx.size() * 8));
  HIP_TRY(d_ebits.ensure(all_bits.size() * 8));
  HIP_TRY(hipMemcpyAsync(d_desc.p, pl.blocks.data(), pl.blocks.size() * sizeof(BlockDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_items.p, pl.items.data(), pl.items.size() * sizeof(Item), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_rank.p, rank.data(), nb, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qvo.p, qv_off.data(), nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qao.p, qa_off.data(), nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_codeo.p, pl.code_off.data(), nb * 8, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_vc.p, vc.data(), vc.size() * sizeof(VarConst), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qv.p, qv.data(), qv.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_qa.p, qa.data(), qa.size(), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(d_codes.p, codes.data(), codes.size(), hipMemcpyHostToDevice, s));
  if (!all_idx.empty()) {
    HIP_TRY(hipMemcpyAsync(d_eidx.p, all_idx.data(), all_idx.size() * 8, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_ebits.p, all_bits.data(), all_bits.size() * 8, hipMemcpyHostToDevice, s));
  }
  HIP_TRY(launch_decode(p.wpad(), p.dtype, d_out, dims, d_desc.as<BlockDesc>(), d_items.as<Item>(),
                        int64_t(pl.items.size()), d_rank.as<uint8_t>(), d_qvo.as<int64_t>(), d_qao.as<int64_t>(),
                        d_codeo.as<int64_t>(), d_vc.as<VarConst>(), d_qv.as<uint8_t>(), d_qa.as<uint8_t>(),
                        d_codes.as<uint8_t>(), s));
  HIP_TRY(launch_scatter(p.dtype, d_out, d_eidx.as<int64_t>(), d_ebits.as<uint64_t>(), int64_t(all_idx.size()), s));
  HIP_TRY(hipStreamSynchronize(s));
  return DLS_OK;
}

}  // extern "C"
