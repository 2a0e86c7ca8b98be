// Launch wrappers of the gfx950 kernels (see dls_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "dls_internal.h"

namespace dls {

// Per-variable constants of the quantizers, computed once on the host so the
// device and any other decoder use identical values.
struct VarConst {
  double eps;       // absolute bound
  double c;         // eps * 2^-16, the lattice step
  double inv_eps;   // 1 / eps
  double inv2eps;   // 1 / (2 eps), the residual quantizer
  float inv_eps_f;  // float(1 / eps), coefficient quantizer
  float pad;
};

struct EscOut {
  unsigned long long* count;  // appended entries (may exceed cap)
  uint64_t* key;              // block << 32 | (t * M_b + p)
  uint64_t* val;              // input value bits
  unsigned long long cap;
};

// How an encode launch finds its work.  Host-driven: `count` items of the
// class list, one workgroup each.  Device-driven (dcount != NULL): a fixed
// grid walks the *dcount items the classifier wrote, so no host round trip
// is needed between the eigensolve and the encode.  An item whose qV or qA
// region would end beyond qv_cap / qa_cap writes nothing and sets
// *overflow (the host then grows the buffers and encodes again).
struct EncodeWork {
  const unsigned int* dcount;
  int64_t count;
  int64_t qv_cap, qa_cap;
  unsigned int* overflow;
};

// Layout of the per-encode counter block: four u64 (escapes, raw blocks,
// warm starts accepted, rejected), kEncodeClasses u32 class counts, the u32
// overflow flag of a device-driven encode, the u32 count of the fallback
// list, the two i64 payload totals (qV bytes, qA bytes), and the Jacobi
// statistics: the u64 count of blocks that reached the sweep cap
// unconverged, then kJacobiSlots u64 partial sums of the sweeps taken (slot
// = workgroup index mod kJacobiSlots, so the atomics spread over addresses).
constexpr int kRankClasses = 6;  // r <= 1, 2, 4, 8, 16, 32
constexpr int kEncodeClasses = 2 * kRankClasses;  // then the same for small slices
constexpr size_t kOverflowAt = 4 * 8 + kEncodeClasses * 4;
constexpr size_t kRejectCountAt = kOverflowAt + 4;  // u32: blocks the warm start left to Jacobi
constexpr size_t kTotalsAt = 88;
constexpr size_t kJacobiAt = kTotalsAt + 16;
constexpr int kJacobiSlots = 64;
constexpr size_t kCounterBytes = kJacobiAt + (1 + kJacobiSlots) * 8;
// sweeps the plain eigensolve takes at most unless the context sets another cap
constexpr int kJacobiMaxSweeps = 12;
// largest slice (points) the small-slice encode takes: its team of lanes x PPT
int encode_small_limit(int wp, int dtype);

// Per-(padded window, element type) entry points of the encode / decode
// kernels (dls_codec.hip, compiled once per pair and part): one rank class of
// the large-slice or the small-slice encode, one rank class of the decode
// (rc < 0: every rank).
#define DLS_CODEC_ENC_DECL(NAME)                                                                                 \
  hipError_t NAME(int rc, const dim3& g, hipStream_t s, const void* F, const Dims& dims, const BlockDesc* desc,  \
                  const Item* items, const int32_t* list, const uint8_t* rank, const double* basis,            \
                  const int64_t* qv_off, const int64_t* qa_off, const int64_t* code_off, const VarConst* vc,   \
                  uint8_t* qv, uint8_t* qa, uint8_t* codes, float* coef, EscOut esc, const EncodeWork& work);
#define DLS_CODEC_DECL(TAG)                                                                                       \
  DLS_CODEC_ENC_DECL(encode_large_##TAG)                                                                          \
  DLS_CODEC_ENC_DECL(encode_small_##TAG)                                                                          \
  hipError_t decode_part_##TAG(int rc, const dim3& g, const dim3& bl, hipStream_t s, void* F, const Dims& dims,   \
                               const BlockDesc* desc, const Item* items, const int32_t* list, const uint8_t* rank, \
                               const int64_t* qv_off, const int64_t* qa_off, const int64_t* code_off,           \
                               const VarConst* vc, const uint8_t* qv, const uint8_t* qa, const uint8_t* codes,  \
                               int64_t count, bool team);
DLS_CODEC_DECL(w16_f32)
DLS_CODEC_DECL(w16_f64)
DLS_CODEC_DECL(w32_f32)
DLS_CODEC_DECL(w32_f64)
#undef DLS_CODEC_DECL
#undef DLS_CODEC_ENC_DECL

// Single-pass encode (k_sketch_basis, k_fused, k_verify in dls_codec.hip)
// for plans whose blocks all span at least one full slice, W <= 16, FP32.
// Per-call state, cleared before the launch: per block a verdict (0 sketch
// basis usable, 1 verified at rank 1, 2 deferred to the two-pass path, 3 no
// usable sketch or rank 1 ruled out by the sketch alone), the list of
// deferred blocks, and u64 counters: payload cursors of the deferred blocks
// (after the rank-1 regions), blocks verified at rank 1, escapes dropped,
// blocks the sketch predicts to fail verification, blocks it rules out.
constexpr int kFusedIters = 6;          // power steps of the sketch's basis after its start column
constexpr int kFusedMinPoints = 1024;   // every block of the plan at least this large
constexpr int kFusedQvCursor = 0, kFusedQaCursor = 1, kFusedAccepted = 2, kFusedDropped = 3, kFusedLikely = 4,
              kFusedPruned = 5, kFusedNCounters = 6;
struct FusedState {
  unsigned int* state;            // [nblocks]
  int32_t* deferred;              // [nblocks]
  unsigned int* ndeferred;        // 1
  unsigned long long* counters;   // kFusedNCounters
};
// r1_off: [nblocks] static qV offsets then [nblocks] static qA offsets of the rank-1 payload
hipError_t launch_sketch_basis(const double* gpart, const int32_t* item_start, const Item* items,
                               const BlockDesc* desc, int64_t nblocks, const double* eps_v, const int64_t* r1_off,
                               uint8_t* rank, double* lam, double* basis, int64_t* qv_size, int64_t* qa_size,
                               int64_t* qv_off, int64_t* qa_off, unsigned int* state, unsigned long long* counters,
                               hipStream_t s);
hipError_t launch_fused(bool bf16, const float* F, const Dims& dims, const BlockDesc* desc,
                        const Item* items, int64_t nitems, const VarConst* vc, double* gpart,
                        const unsigned int* state, const double* basis, const int64_t* qv_off, const int64_t* qa_off,
                        const int64_t* code_off, uint8_t* qv, uint8_t* qa, uint8_t* codes, float* coef, EscOut esc,
                        hipStream_t s);
hipError_t launch_verify(const double* gpart, const int32_t* item_start, const BlockDesc* desc, int64_t nblocks,
                         const double* eps_v, const double* basis, double* lam, const FusedState& fs, hipStream_t s);
hipError_t launch_fix_escapes(uint64_t* key, const unsigned long long* count, unsigned long long cap,
                              const unsigned int* state, unsigned long long* ndropped, hipStream_t s);
// payload offsets of the deferred blocks: base + a bump cursor
hipError_t launch_alloc_deferred(const int32_t* list, const unsigned int* count, int64_t nmax, const int64_t* qv_size,
                                 const int64_t* qa_size, unsigned long long* counters, int64_t qv_base,
                                 int64_t qa_base, int64_t* qv_off, int64_t* qa_off, hipStream_t s);

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
// totals[0] = qv_off[n-1] + qv_size[n-1], totals[1] likewise for qA
hipError_t launch_totals(const int64_t* qv_off, const int64_t* qv_size, const int64_t* qa_off,
                         const int64_t* qa_size, int64_t n, int64_t* totals, hipStream_t s);

// Slices of at most kSmallSlice points may share workgroups (one wave each)
// when the plan is split into these two lists of slice indices.
constexpr int kSmallSlice = 256;
struct GramSplit {
  const int32_t* large;
  int64_t nlarge;
  const int32_t* small;
  int64_t nsmall;
};
hipError_t launch_gram(int wp, int dtype, bool bf16, const void* F, const Dims& dims, const BlockDesc* desc,
                       const Item* items, int64_t nitems, const GramSplit* split, double* gpart, hipStream_t s);
// list (may be NULL): solve only the *list_count blocks list[0..) (a
// device-written list; the grid covers nblocks, the rest exits at once).
// At most max_sweeps sweeps per block; jstats (the Jacobi statistics of the
// counter block) is added to.
hipError_t launch_eigen(int wp, const double* gpart, const int32_t* item_start, const BlockDesc* desc,
                        int64_t nblocks, const double* eps_v, int r_max, uint8_t* rank, double* lam,
                        double* basis, int64_t* qv_size, int64_t* qa_size, unsigned long long* nraw,
                        const int32_t* list, const unsigned int* list_count, unsigned long long* jstats,
                        int max_sweeps, hipStream_t s);
// list of the blocks b < n with flag[b] != 0, in any order; *count is added to
hipError_t launch_compact_flags(const uint8_t* flag, int64_t n, int32_t* list, unsigned int* count, hipStream_t s);
// learned warm start (dls_learned.hip)
// Feature rows are computed per list: blocks of at most kFeatSmall points
// (16 lanes each), the other blocks of at most kWarmMaxPoints points (one
// wavefront each), and the rest (zero rows).
constexpr int kFeatSmall = 16;
struct FeatureLists {
  const int32_t* small;
  int64_t nsmall;
  const int32_t* wave;
  int64_t nwave;
  const int32_t* zero;
  int64_t nzero;
};
hipError_t launch_features(int dtype, const void* F, const Dims& dims, const BlockDesc* desc,
                           const FeatureLists& lists, const double* eps_v, float* feat, hipStream_t s);
hipError_t launch_normalize(const float* raw, int64_t n, const float* norm, float* z, hipStream_t s);
hipError_t launch_gemm(bool ta, bool tb, bool bf16, const float* A, int lda, const float* B, int ldb, float* C,
                       int ldc, int M, int N, int K, const float* bias, int relu, hipStream_t s);
hipError_t launch_loss(const float* out, const int32_t* rank, const float* basis, const int32_t* wb, int64_t n,
                       float* gout, float* loss, hipStream_t s);
hipError_t launch_colsum(const float* G, int64_t n, int cols, float* out, hipStream_t s);
hipError_t launch_relu_mask(float* dh, const float* h, int64_t n, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float c1, float c2,
                       hipStream_t s);
// Blocks of more points than this take the plain eigensolve: the warm start
// pays for one extra read of the block (its features), which outweighs the
// Jacobi work it saves beyond about this size at W = 16.
constexpr int kWarmMaxPoints = 256;

// Warm-start network 80 -> 128 -> 128 -> 272 (ReLU), flat FP32 parameters
// W1 (80 x 128, row-major [in][out]), b1, W2, b2, W3, b3.
constexpr int kNF = 80, kH = 128, kNO = 272;
constexpr int64_t kOffW1 = 0, kOffb1 = 80 * 128, kOffW2 = kOffb1 + 128, kOffb2 = kOffW2 + 128 * 128,
                  kOffW3 = kOffb2 + 128, kOffb3 = kOffW3 + 128 * 272, kNParam = kOffb3 + 272;

// Inference forward of the network, the three layers fused (bf16 products,
// FP32 accumulation, bit-identical to the layer-by-layer path).  `packed`
// holds the weights as written by launch_pack_weights.
constexpr int kPackLd = kH + 4;  // bf16 leading dimension of a packed layer ([out][in])
constexpr int64_t kPackedWeightBytes = int64_t(2) * kPackLd * (kH + kH + kNO);
hipError_t launch_pack_weights(const float* P, short* packed, hipStream_t s);
hipError_t launch_mlp_forward(const float* raw, int64_t n, const float* norm, const float* P, const short* packed,
                              float* out, hipStream_t s);
hipError_t launch_warmstart(const double* gpart, const int32_t* item_start, const BlockDesc* desc, int64_t nblocks,
                            const double* eps_v, int r_max, const float* mlp_out, int iters, int margin,
                            uint8_t* rank, double* lam, double* basis, int64_t* qv_size, int64_t* qa_size,
                            uint8_t* reject, unsigned long long* counters, unsigned long long* jstats,
                            hipStream_t s);
hipError_t launch_scan(const int64_t* in, int64_t n, int64_t* out, int64_t* tmp, hipStream_t s);
// L2 / NRMSE-bounded mode (dls_l2.hip).  Per block: rank byte (kL2Raw =
// values stored verbatim), coefficient step, budget; the squared error of
// every slice; payload regions as in the absolute mode (qV, qA planes; a
// raw block's values in its qA region).
constexpr int kL2Raw = 255;
// Global-basis mode (dls_global.hip).  Per variable an M x M basis Phi[i][s]
// (FP64 values on the 2^-24 grid); per patch-snapshot a coefficient count
// (0xFFFF = raw), a step exponent and a slot of 8 M bytes (kept indices u16
// at 0, coefficients int32 at 4 M, or the raw values) compacted afterwards.
constexpr int kGbParts = 256;
// partial sums per variable of the field's sum of squares (enough
// workgroups to keep HBM busy; the partials are added in a fixed order)
constexpr int kGbSumParts = 2048;
constexpr int kGbRaw = 0xFFFF;
constexpr int kGbMaxM = 1024;
hipError_t launch_gb_budget(int dtype, const void* F, int64_t per_var, int nvars, const double* target,
                            double* part, double* cv, hipStream_t s);
hipError_t launch_gb_samples(int dtype, const void* F, const Dims& dims, int var, int px, int py, int pz, int kind,
                             uint64_t s0, int64_t S, double* Q, hipStream_t s);
hipError_t launch_gb_gram(const double* Q, int64_t S, int M, int Mp, double* G, hipStream_t s);
hipError_t launch_gb_eye(double* V, int Mp, hipStream_t s);
hipError_t launch_gb_jacobi_round(const double* Ain, double* Aout, double* V, int Mp, int round, hipStream_t s);
constexpr int kGbMaxSweeps = 40;
hipError_t launch_gb_jacobi_lds(const double* G, int Mp, double floor2, int max_sweeps, double* A, double* V,
                                int* info, hipStream_t s);
hipError_t launch_gb_offnorm(const double* A, double* Acopy, int Mp, double* part, double* out, hipStream_t s);
hipError_t launch_gb_finish(const double* A, const double* V, int M, int Mp, double* Phi, hipStream_t s);
hipError_t launch_gb_cosine(int px, int py, int pz, double* Phi, hipStream_t s);
hipError_t launch_gb_project(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nb0,
                             int64_t nb1, const double* phi, int px, int py, int M, double* alpha, hipStream_t s);
hipError_t launch_gb_select(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nblocks,
                            const double* phi, const double* cv, const double* alpha, int px, int py, int M,
                            int32_t* count, int32_t* kexp, uint8_t* slot, int32_t* n0, hipStream_t s);
hipError_t launch_gb_patch64(int dtype, const void* F, const Dims& dims, const BlockDesc* desc, int64_t nb0,
                             int64_t nb1, const double* phi, const double* cv, int px, int py, int M, int32_t* count,
                             int32_t* kexp, uint8_t* slot, int32_t* n0, hipStream_t s);
hipError_t launch_gb_sizes(const BlockDesc* desc, int64_t nblocks, const int32_t* count, int esize, int64_t* nidx,
                           int64_t* nraw, unsigned long long* raw_patches, hipStream_t s);
hipError_t launch_gb_compact(const BlockDesc* desc, int64_t nblocks, int M, const int32_t* count, const uint8_t* slot,
                             const int64_t* idx_off, const int64_t* raw_off, int esize, uint16_t* idx_out,
                             int32_t* q_out, uint8_t* raw_out, hipStream_t s);
hipError_t launch_gb_decode(int dtype, void* F, const Dims& dims, const BlockDesc* desc, int64_t nblocks,
                            int nvars, const double* phi, int px, int py, int M, const int32_t* count,
                            const int32_t* kexp, const int64_t* idx_off, const int64_t* raw_off,
                            const uint16_t* idx, const int32_t* q, const uint8_t* raw, hipStream_t s);
hipError_t launch_l2_gram(int wp, int dtype, const void* F, const Dims& dims, const BlockDesc* desc,
                          const Item* items, int64_t nitems, double* gpart, double* fsq, hipStream_t s);
// range: per variable its slice range [range[2v], range[2v + 1]); part:
// 256 partial sums per variable
hipError_t launch_l2_budget(const double* fsq, const int64_t* range, double* part, const double* target,
                            int64_t per_var, int nvars, double* cv, double* eig_eps, hipStream_t s);
hipError_t launch_l2_params(const BlockDesc* desc, int64_t nblocks, const double* lam, int wp,
                            const uint8_t* eig_rank, const double* cv, bool first, int esize, uint8_t* l2rank,
                            double* step, double* e2, int64_t* qv_size, int64_t* qa_size, hipStream_t s);
hipError_t launch_l2_encode(int wp, int dtype, const void* F, const Dims& dims, const BlockDesc* desc,
                            const Item* items, int64_t nitems, const uint8_t* l2rank, const double* step,
                            const double* basis, const int64_t* qv_off, const int64_t* qa_off, uint8_t* qv,
                            uint8_t* qa, uint8_t* overflow, double* errp, hipStream_t s);
hipError_t launch_l2_check(const BlockDesc* desc, const int32_t* item_start, int64_t nblocks, const double* errp,
                           const double* e2, const uint8_t* overflow, int rcap, uint8_t* l2rank, double* berr,
                           unsigned int* nfail, hipStream_t s);
hipError_t launch_l2_decode(int wp, int dtype, void* F, const Dims& dims, const BlockDesc* desc, const Item* items,
                            int64_t nitems, const uint8_t* l2rank, const double* step, const int64_t* qv_off,
                            const int64_t* qa_off, const uint8_t* qv, const uint8_t* qa, hipStream_t s);
// Allocation-free range: the partials live in a fixed device array (one per
// GPU) whose address range_scratch() returns for the current device;
// results at scratch_ptr + nvars * 2 * 1024 as (min, max) per variable.
constexpr int kRangeNoAllocVars = 64;
constexpr int kRangeParts = 1024;  // partials per variable (fewer for short fields)
hipError_t range_scratch(int device, double** scratch_ptr);
hipError_t launch_range_noalloc(double* scratch_ptr, int dtype, const void* F, int nvars, int64_t n_per_var,
                                hipStream_t s);
hipError_t launch_range(int dtype, const void* F, int nvars, int64_t n_per_var, double* part, int nparts,
                        double* out, hipStream_t s);
// skip (may be NULL): items of blocks with skip[block] == 1 are left out
hipError_t launch_classify(const Item* items, int64_t nitems, const uint8_t* rank, int small_limit,
                           unsigned int* counts, int32_t* lists, hipStream_t s, const unsigned int* skip = nullptr);
hipError_t launch_encode(int wp, int dtype, int cls, const void* F, const Dims& dims, const BlockDesc* desc,
                         const Item* items, const int32_t* list, const EncodeWork& work, const uint8_t* rank,
                         const double* basis, const int64_t* qv_off, const int64_t* qa_off,
                         const int64_t* code_off, const VarConst* vc, uint8_t* qv, uint8_t* qa,
                         uint8_t* codes, float* coef, EscOut esc, hipStream_t s);
hipError_t launch_decode(int wp, int dtype, void* F, const Dims& dims, const BlockDesc* desc,
                         const Item* items, int64_t nitems, const uint8_t* rank, const int64_t* qv_off,
                         const int64_t* qa_off, const int64_t* code_off, const VarConst* vc,
                         const uint8_t* qv, const uint8_t* qa, const uint8_t* codes, hipStream_t s);
hipError_t launch_scatter(int dtype, void* F, const int64_t* idx, const uint64_t* bits, int64_t n,
                          hipStream_t s);
// decode of the `count` items of one rank class (the encode's class list;
// small: a small-slice class, decoded by one wavefront per slice)
hipError_t launch_decode_class(int wp, int dtype, int rc, bool small, const int32_t* list, int64_t count, void* F,
                               const Dims& dims, const BlockDesc* desc, const Item* items, const uint8_t* rank,
                               const int64_t* qv_off, const int64_t* qa_off, const int64_t* code_off,
                               const VarConst* vc, const uint8_t* qv, const uint8_t* qa, const uint8_t* codes,
                               hipStream_t s);
// escapes from the encoder's (key, value bits) list
hipError_t launch_scatter_keys(int dtype, void* F, const Dims& dims, const BlockDesc* desc, const uint64_t* key,
                               const uint64_t* bits, int64_t n, hipStream_t s);

struct PlanScratch;
PlanScratch* plan_scratch_new();
void plan_scratch_delete(PlanScratch* s);
// Adaptive leaves and split bits of every variable (see dls_plan.hip).
hipError_t adaptive_plan(const Problem& p, const void* F, hipStream_t s, PlanScratch& scratch, Plan& plan,
                         std::string& err);

}  // namespace dls
