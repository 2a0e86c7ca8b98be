/*
 * dls.h -- C ABI of libdls, the MI355X (gfx950) encoder/decoder of
 * Discontinuous DLS (data-informed local subspaces), an error-bounded lossy
 * compressor for structured-grid fields.
 *
 * The problem statement follows Alg. 1 of the paper (inputs: snapshots, patch
 * size, target error; outputs: coefficients and the orthonormal basis) and
 * Alg. 2 (the inverse), extended with a time window and an absolute
 * pointwise error bound per variable:
 *
 *   for every spatial patch x time window (a "block") the library gathers the
 *   snapshot matrix X (W_b x M_b), forms its Gram product X X^T (the
 *   cross-product SVD of Sec. 2.7.1), eigensolves it for a local basis
 *   (Sec. 2.3, Eqs. (2)-(3)), truncates it to the smallest rank r whose
 *   discarded energy meets the local tolerance (Sec. 2.4 Eq. (4), Sec. 2.5
 *   Eq. (6)), projects (Eq. (5)), quantizes basis and coefficients (the
 *   bit-grooming step of Sec. 2.5), reconstructs on an integer lattice and
 *   quantizes the pointwise residual so that every returned value lies
 *   within abs_eps[v] of the input.  Batches of 1000 blocks are deflated on
 *   host threads (gzip's algorithm, Sec. 2.5) behind an addressable header
 *   (Sec. 2.7.2).
 *
 * Conventions shared by every entry point:
 *   - Every call returns a dls_status; 0 is success.  No C++ exception
 *     crosses the ABI.  On failure dls_last_error() describes the cause.
 *   - Field layout: F[var][t][z][y][x], x fastest, contiguous, on the device;
 *     element type float (DLS_F32) or double (DLS_F64).  2D fields use nz = 1
 *     and pz = 1.
 *   - A `stream` argument is a hipStream_t (NULL = the default stream),
 *     owned by the caller.  Calls are synchronous: they return after their
 *     device work on that stream has completed.
 *   - Device pointers are owned by the caller unless stated otherwise.
 *   - Not thread-safe on the same dls_ctx; distinct contexts may be used
 *     concurrently from different host threads.
 */
#ifndef DLS_H
#define DLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  DLS_OK = 0,
  DLS_EINVAL = -1,       /* invalid argument; nothing was written           */
  DLS_ENOMEM = -2,       /* host or device allocation failed                */
  DLS_EDEVICE = -3,      /* a HIP call or kernel launch failed              */
  DLS_ECORRUPT = -4,     /* stream truncated or inconsistent                */
  DLS_EUNSUPPORTED = -5  /* valid request this build does not implement     */
} dls_status;

typedef enum { DLS_F32 = 0, DLS_F64 = 1 } dls_dtype;

/* Operand precision of the Gram contraction (Sec. 2.2's eigenbasis).
 * DLS_PREC_BF16 rounds the snapshots to bfloat16 as the matrix cores take
 * them (FP32 accumulation per 64-point chunk, FP64 across chunks); the
 * eigenbasis then carries bfloat16-level error.  The projection, the
 * eigensolve, the lattice reconstruction and the bound check use the
 * stored values in every mode, so the bound holds exactly either way. */
typedef enum { DLS_PREC_FP32 = 0, DLS_PREC_BF16 = 1 } dls_precision;

/* dls_params.flags */
enum {
  DLS_ADAPTIVE = 1,  /* quadtree (2D) / octree (3D) patches between pmin and
                        px, computed per variable from snapshot 0: a node
                        of edge e > pmin splits into its half-edge children
                        while its mean gradient magnitude exceeds the 80th
                        percentile sorted(g)[floor(0.8 (n-1))]             */
  DLS_LEARNED = 2,   /* warm-started eigensolve with the model attached by
                        dls_ctx_set_model (window <= 16); blocks whose
                        prediction fails the rank test fall back to Jacobi */
  DLS_PERSISTENT = 4, /* batched launch.  Plans whose blocks all span at
                        least 1024 points (FP32, window <= 16): one fused
                        persistent launch reads every slice once into
                        registers, forms its Gram, and the slice that
                        completes a block solves it at rank 1 when the
                        exact discarded energy of a power-iteration basis
                        meets the tolerance (Sec. 2.4 Eq. (4)); the block
                        is then encoded from registers, without a second
                        read of the field.  Blocks that need a higher rank
                        take the Jacobi eigensolve and a second read; when
                        the first slice of more than half the blocks
                        already predicts that, the call runs two-pass.
                        Other plans of up to 65536 slices: no host round
                        trip between the eigensolve and the encode (the
                        encode kernels walk device-written rank-class
                        lists); larger plans keep the host-driven launch.
                        Payload buffers are sized by earlier calls; when
                        they do not fit, the library grows them and encodes
                        the call again two-pass.  The stream decodes to
                        the same guarantees; its rank-1 bases come from the
                        power iteration instead of Jacobi. */
  DLS_L2 = 8,        /* L2 / NRMSE-bounded mode, the paper's error control
                        (Sec. 2.4: global budget eps_t ||u||, Eq. (4)
                        equal-share local tolerance; Alg. 1 step 3: fewest
                        coefficients meeting it).  abs_eps[v] is then the
                        target NRMSE of variable v as a fraction (0.01 =
                        1 %).  Each block gets the budget e2 = eps_t^2
                        ||u_v||^2 M_b W_b / K_v (K_v values of the
                        variable), the smallest rank whose eigenvalue tail
                        fits 0.36 e2, coefficients quantized with step
                        0.4 sqrt(e2 / (r M_b)) and a 2^-24 basis grid, and
                        the exact error of the decoded values is checked:
                        a block above e2 is encoded again one rank higher,
                        or stored verbatim.  No residual codes.  Every
                        variable's NRMSE is within its target.  The Gram is
                        FP64 in this mode (precision has no effect): the
                        rank test resolves tails of ~1e-8 of a block's
                        energy at tight targets.  Not with DLS_LEARNED;
                        DLS_PERSISTENT has no effect. */
  DLS_GLOBAL = 16    /* the paper's global-basis method (Sec. 2.2-2.5,
                        Alg. 1): one M x M basis per variable (M = px py pz
                        <= 1024, px <= nx, py <= ny, pz <= nz) learned once
                        (dls_params.basis), applied to every patch of every
                        snapshot (window must be 1).  DLS_BASIS_SVD: S = 4M
                        patches of snapshot 0 at SplitMix64 positions
                        (state seed + v, three draws per patch: x0, y0, z0
                        modulo their ranges) form Q; the full eigenbasis of
                        Q^T Q, eigenvalues descending, canonical signs
                        (Eqs. (2)-(3), no truncation).  DLS_BASIS_COSINE /
                        DLS_BASIS_RANDOM: the orthonormal DCT-II tensor
                        basis / the eigenbasis of an M x M matrix of
                        uniform [-1, 1) SplitMix64 draws (Sec. 4's study).
                        The basis is stored on the 2^-24 grid.  abs_eps[v]
                        is the NRMSE target as in DLS_L2; a patch of one
                        snapshot gets e2 = eps_t^2 ||u_v||^2 M_b / K_v and
                        keeps the fewest coefficients alpha = Phi^T u in
                        decreasing |alpha| (ties: lower index) whose
                        dropped energy is <= 0.36 e2 (Eq. (6)), groomed to
                        the grid 2^floor(log2(0.4 sqrt(e2 / n))); the exact
                        error of the decoded values must be <= e2, else one
                        more coefficient, and the patch is stored verbatim
                        past n = M.  Edge patches are zero-padded.  Not with
                        DLS_ADAPTIVE, DLS_LEARNED or DLS_L2; precision and
                        DLS_PERSISTENT have no effect.  Device memory:
                        16 B per value beyond the field (coefficients and
                        per-patch slots). */
};

/* dls_params.basis (DLS_GLOBAL) */
typedef enum { DLS_BASIS_SVD = 0, DLS_BASIS_COSINE = 1, DLS_BASIS_RANDOM = 2 } dls_basis_kind;

struct dls_model;

typedef struct dls_params {
  uint32_t struct_size;    /* = sizeof(dls_params); ABI versioning          */
  int32_t nvars;           /* variables, >= 1                               */
  int64_t nx, ny, nz, nt;  /* grid (x fastest) and time steps, all >= 1     */
  int32_t dtype;           /* dls_dtype                                     */
  int32_t px, py, pz;      /* patch edge (uniform) or largest leaf edge
                              (DLS_ADAPTIVE: px = py = pz (2D: pz = 1),
                              power of two); 1..32, pz = 1 when nz = 1      */
  int32_t pmin;            /* smallest leaf edge (DLS_ADAPTIVE), power of 2 */
  int32_t window;          /* W: time steps per window, 1..32; the last
                              window is truncated                           */
  int32_t r_max;           /* rank cap, 0 -> min(window, 32)                */
  int32_t precision;       /* dls_precision                                 */
  uint32_t flags;          /* DLS_ADAPTIVE | DLS_LEARNED | DLS_PERSISTENT |
                              DLS_L2 | DLS_GLOBAL                           */
  const double* abs_eps;   /* host array of nvars absolute bounds, each
                              finite and > 0; read during the call only    */
  int32_t basis;           /* DLS_GLOBAL: dls_basis_kind                    */
  uint64_t seed;           /* DLS_GLOBAL: state of the learning draws       */
  struct dls_model* model; /* DLS_LEARNED in dls_compress: the warm-start
                              model (dls_model_create / dls_model_set);
                              NULL otherwise.  Not owned; must outlive the
                              call.  The context API takes it through
                              dls_ctx_set_model instead (this field is
                              ignored by dls_encode).                        */
  int32_t warm_iters;      /* with model: subspace iterations, 0 -> 2       */
  int32_t rank_margin;     /* with model: predicted-rank margin, 0..8       */
} dls_params;

/* Per-call results of dls_encode, in device memory owned by the context
 * (valid until the next dls_encode on it or dls_ctx_destroy).  Offsets are
 * in bytes into the named buffers.  Diagnostics for tests and benchmarks. */
typedef struct dls_encode_info {
  int64_t nblocks;          /* blocks: variable, then window, then patch    */
  int64_t nescapes;         /* escaped points (stored verbatim)             */
  int64_t nraw;             /* raw blocks (non-finite input)                */
  int64_t wpad;             /* 16 or 32: padded Gram order                  */
  const uint8_t* d_rank;    /* [nblocks] rank r (0 = raw block)             */
  const double* d_lam;      /* [nblocks][wpad] eigenvalues of X X^T, desc   */
  const double* d_basis;    /* [nblocks][wpad][wpad] eigenvectors, column k
                               at [k][t], canonical signs                   */
  const int32_t* d_desc;    /* [nblocks][8] x0, y0, z0, t0, extents (px | py<<8 |
                               pz<<16 | w<<24), var, M_b, vector flag      */
  int64_t qa_bytes, codes_bytes;  /* payload bytes (DLS_GLOBAL: 6 per kept
                               coefficient -- index and value -- plus the raw
                               patches' values; codes_bytes 0)               */
  const uint8_t* d_qa;      /* qA planes, per block at d_qa_off[b]          */
  const uint8_t* d_codes;   /* residual codes, one byte per value (zigzag  */
                            /* int8, 0xFF = escape), per block at d_code_off */
  const int64_t* d_qa_off;  /* [nblocks]                                    */
  const int64_t* d_code_off;/* [nblocks]                                    */
  const float* d_coef;      /* [sum M_b r_b] FP32 coefficients A[k][p] at
                               d_qa_off[b]/4 when requested, else NULL      */
  int64_t nwarm_accept;     /* DLS_LEARNED: blocks solved by the warm start  */
  int64_t nwarm_reject;     /* DLS_LEARNED: blocks that fell back to Jacobi   */
  double gpu_ms;            /* device time of the whole encode (HIP events) */
  double stage_ms[5];       /* HIP-event time of each stage on the caller's
                               stream: plan (adaptive: gradient, percentile,
                               node sums, tree walk, upload), Gram,
                               eigensolve + rank, offset scan + rank classes,
                               projection / quantization / residual codes;
                               in the fused single pass: the fused kernel,
                               Jacobi of the deferred blocks, their payload
                               regions and slice lists, their encode        */
  int64_t nfast_accept;     /* fused single pass: blocks solved at rank 1 and
                               encoded in the same pass                      */
  int64_t ndeferred;        /* fused single pass: blocks left to the Jacobi
                               eigensolve and a second read                 */
  int32_t launch_mode;      /* 0 host-driven, 1 device-driven, 2 fused single
                               pass (see DLS_PERSISTENT)                     */
  int64_t jacobi_sweeps;    /* sweeps the plain eigensolve took, summed over
                               the blocks it solved; one sweep of order wpad
                               costs 9 wpad^2 (wpad - 1) FP64 flops          */
  int64_t jacobi_unconverged; /* blocks (and warm-start Rayleigh-Ritz solves)
                               that used every sweep of the cap without off(A)
                               <= 1e-13 ||A|| before one of them: their basis
                               is orthonormal, their eigenvalues (so their
                               rank) may not be converged; the bound holds
                               regardless                                   */
  double jacobi_ms;         /* HIP-event time of the Jacobi launch alone      */
  double fused_ms;          /* fused single pass: HIP-event time of the fused
                               kernel alone (0 otherwise)                    */
  int64_t npredicted_deferred; /* DLS_PERSISTENT plans of large FP32 blocks:
                               blocks whose sketch predicts that the rank-1
                               basis fails on the whole block               */
  int64_t npruned;          /* of those, blocks where the sketch alone proves
                               it (its discarded energy exceeds tau)         */
  int32_t fused_declined;   /* 1: more than half the blocks were predicted to
                               fail, so the call ran two-pass                */
  int32_t l2_passes;        /* DLS_L2: encode passes (1 when every block met
                               its budget at the rank its eigenvalues gave)  */
} dls_encode_info;

typedef struct dls_ctx dls_ctx;

/* Create / destroy an encoder context holding device workspace, reused
 * across calls with the same parameters.  `device` is the HIP device
 * ordinal the context's memory lives on. */
dls_status dls_ctx_create(int device, dls_ctx** out);
void dls_ctx_destroy(dls_ctx* ctx);

/* Launch strategy of DLS_PERSISTENT plans that do not take the single pass:
 * plans of at most device_driven_max_items slices take the device-driven
 * encode (no host round trip between the eigensolve and the encode, the
 * encode kernels walk device-written rank-class lists); larger plans the
 * host-driven one (one launch per rank class sized from a readback).  The
 * two write identical streams; which is faster depends on the plan (the
 * device-driven launch's looping workgroups are slower on very long lists).
 * Default 65536; 0 always host-driven.  The autotuner of the Python package
 * (paper_2601_20113_amd.autotune) times the choices on a workload and caches
 * the fastest.  DLS_EINVAL on a negative count. */
dls_status dls_ctx_set_launch(dls_ctx* ctx, int64_t device_driven_max_items);

/* Graph replay (enabled by default; 0 launches every kernel on its own,
 * with identical results):
 *  - the device-driven encode (see dls_ctx_set_launch): after an eager call
 *    the sequence from the Gram to the encode is captured on a stream of
 *    the context and replayed on the caller's stream by later calls while
 *    the field pointer, the problem, every workspace buffer, the model and
 *    its parameters and the launch shapes are unchanged (otherwise the call
 *    runs eagerly and captures again); the replay's stages are not timed
 *    separately (dls_encode_info.stage_ms counts it as the encode stage);
 *  - the global basis's Jacobi sweeps (DLS_GLOBAL, bases of order > 64):
 *    one sweep's M - 1 rotation rounds and norm kernels, replayed per sweep.
 * DLS_EINVAL unless enabled is 0 or 1. */
dls_status dls_ctx_set_graphs(dls_ctx* ctx, int enabled);

/* Cap on the sweeps of the plain Jacobi eigensolve (Sec. 2.7.1: the basis
 * is the eigenvector set of the block's Gram) for later encodes in this
 * context; default 12, which the tested workloads never reach.  A lower cap
 * trades eigenvalue accuracy (and with it the rank choice) for time; the
 * pointwise bound still holds since the residual codes correct any
 * orthonormal basis.  Blocks that stop at the cap are counted in
 * dls_encode_info.jacobi_unconverged.  Errors: DLS_EINVAL (NULL context,
 * max_sweeps outside [1, 64]). */
dls_status dls_ctx_set_jacobi_sweeps(dls_ctx* ctx, int max_sweeps);

/* Device half of compression (Alg. 1 step 3 for every block): plan, Gram,
 * eigensolve, rank, projection, quantization, lattice reconstruction,
 * residual codes and escapes, leaving the packed payload in the context's
 * device buffers.  d_field: device pointer to the field (layout above).
 * keep_coef != 0 also stores the FP32 coefficients A for diagnostics.
 * Errors: DLS_EINVAL (params), DLS_ENOMEM, DLS_EDEVICE. */
dls_status dls_encode(dls_ctx* ctx, const void* d_field, const dls_params* p,
                      void* stream, int keep_coef);

/* Per-variable value range of a device field (layout above; nvars variables
 * of values_per_var = nt*nz*ny*nx elements each), computed on the device in
 * FP64 with non-finite values skipped.  The absolute bound of the benchmark
 * configurations is eps_v = c * (max_v - min_v).  min_out / max_out: host
 * arrays of nvars doubles (+inf / -inf for a variable with no finite value).
 * Errors: DLS_EINVAL, DLS_ENOMEM, DLS_EDEVICE. */
dls_status dls_range(const void* d_field, int32_t nvars, int64_t values_per_var, int32_t dtype,
                     void* stream, double* min_out, double* max_out);

/* dls_range without any device allocation, for callers that cannot
 * allocate (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments and results as dls_range, bitwise.
 * Its partial minima / maxima live in a fixed device array of the library
 * (about 1 MiB, one copy per GPU, held until the process ends) instead of
 * buffers allocated per call; the device is the current one.  At most 64
 * variables (DLS_EINVAL above that, nothing launched).  Calls on one GPU
 * share that array: calls that overlap on one GPU (other host threads, or
 * work still queued on another stream) race, so serialise them.  Errors:
 * DLS_EINVAL, DLS_EDEVICE. */
dls_status dls_range_noalloc(const void* d_field, int32_t nvars, int64_t values_per_var, int32_t dtype,
                             void* stream, double* min_out, double* max_out);

/* Diagnostics of the last dls_encode on ctx (pointers into ctx memory). */
dls_status dls_encode_info_get(const dls_ctx* ctx, dls_encode_info* info);

/* Host half of compression: copy the payload of the last dls_encode to host,
 * deflate each batch of 1000 blocks on host threads and write the stream
 * (header, per-batch offset table, zlib streams; Sec. 2.7.2).  *out is a
 * library-owned host buffer; release it with dls_free. */
dls_status dls_finalize(dls_ctx* ctx, uint8_t** out, size_t* out_bytes);

/* Device half of decompression (Alg. 2, Eq. (7)) for the last dls_encode of
 * this context: reconstructs every value from the context's device payload
 * (quantized basis and coefficients, residual codes, escapes) into d_out, a
 * caller-owned device buffer laid out like the encoded field
 * ([var][t][z][y][x], the encode's dtype, nvars * nt * nz * ny * nx values).
 * The result is bitwise the one dls_decompress gives for the stream
 * dls_finalize writes.  Enqueued on `stream` (a hipStream_t, NULL = default
 * stream); the call returns without waiting, and the context must not be
 * encoded again before the stream has reached this point.  out_bytes is the
 * size of d_out in bytes.  DLS_EINVAL (nothing written) when an argument is
 * NULL, the context holds no encode result, or out_bytes is below
 * nvars * nt * nz * ny * nx * element size of the last encode. */
dls_status dls_decode(dls_ctx* ctx, void* d_out, size_t out_bytes, void* stream);

/* dls_encode + dls_finalize with a temporary context. */
dls_status dls_compress(const void* d_field, const dls_params* p, void* stream,
                        uint8_t** out, size_t* out_bytes);

/* Read the header of a stream (host buffer in[0..in_bytes)): the
 * addressable header of Sec. 2.7.2 (problem statement, per-variable bounds,
 * adaptive split bits, one (offset, size) entry per batch of 1000 blocks).
 * Writes the problem statement to *p_out (abs_eps is set to NULL; flags
 * carry DLS_ADAPTIVE / DLS_L2 / DLS_GLOBAL, basis the global basis kind),
 * the bounds (or NRMSE targets) to eps_out[0..min(nvars, eps_cap)) when
 * eps_out is not NULL, and the block count (patch-snapshots in the global
 * mode) to *nblocks when not NULL.  The bounds and the count are separate
 * outputs because dls_params holds a pointer to caller-owned bounds.  No
 * device work.  DLS_ECORRUPT on a bad header, DLS_EINVAL on a NULL p_out. */
dls_status dls_query(const uint8_t* in, size_t in_bytes, dls_params* p_out,
                     double* eps_out, int32_t eps_cap, int64_t* nblocks);

/* Alg. 2: inflate every batch, rebuild the lattice values of every block,
 * apply the escapes and assemble the field (Eq. (7)) into d_field_out, a
 * caller-allocated device buffer of nvars*nt*nz*ny*nx elements of the
 * stream's dtype.  DLS_ECORRUPT on a truncated or inconsistent stream. */
dls_status dls_decompress(const uint8_t* in, size_t in_bytes, void* d_field_out,
                          void* stream);

/* Summary of a stream, computed on the host (no device work): every batch
 * of Sec. 2.7.2 is inflated and its per-block sections read.  Counts that
 * only the encoder knows (warm starts accepted, Jacobi fallbacks and sweeps)
 * are not in the stream; dls_encode_info reports them.  DLS_ECORRUPT on a
 * truncated or inconsistent stream. */
typedef struct dls_stream_stats {
  int64_t nblocks, nbatches, nraw, nescapes;
  int64_t rank_hist[33];     /* rank_hist[r] = blocks with rank r (global
                                mode: patches keeping r coefficients, 32 for
                                32 or more)                                 */
  int64_t payload_bytes;     /* uncompressed payload                        */
  int64_t stream_bytes;      /* whole stream                                */
} dls_stream_stats;
dls_status dls_stats(const uint8_t* in, size_t in_bytes, dls_stream_stats* s);

/* ---- learned warm start ------------------------------------------------
 * A small network (80 inputs -> 128 -> 128 -> 272 outputs, ReLU) maps the
 * statistics of one block (dls_features) to 16 rank logits and a 16 x 16
 * starting basis (outputs 16 + 16 k + t = V0[t][k]).  The encode path with
 * DLS_LEARNED runs `iters` steps of subspace iteration from the first rhat
 * predicted columns, a Rayleigh-Ritz step, and keeps the smallest rank whose
 * discarded energy meets the local tolerance (Sec. 2.4 Eq. (4)); otherwise
 * the block falls back to the Jacobi eigensolve.  Training runs on the GPU:
 * forward and backward products on the matrix cores (bf16 operands, FP32
 * accumulation), loss = cross entropy of the rank + masked squared error of
 * the basis columns k < r, t < W_b, Adam (lr, 0.9, 0.999, 1e-8).
 *
 * Parameters are one FP32 vector of DLS_MODEL_NPARAM values, row-major:
 * W1 (80 x 128), b1 (128), W2 (128 x 128), b2 (128), W3 (128 x 272), b3 (272);
 * the normalisation is 32 values: mean and standard deviation of the 16
 * statistics (the 64 pooled inputs are already normalised). */
#define DLS_MODEL_NPARAM 61968
#define DLS_NFEAT 80
#define DLS_NOUT 272
typedef struct dls_model dls_model;  /* declared above as struct dls_model */
/* Create a model on `device` with all parameters zero and identity
 * normalisation; set them with dls_model_set. */
dls_status dls_model_create(int device, dls_model** out);
void dls_model_destroy(dls_model* m);
/* Copy parameters (and, if norm != NULL, the 32 normalisation values) from
 * host arrays; resets the Adam state.  DLS_EINVAL on NULL params. */
dls_status dls_model_set(dls_model* m, const float* params, const float* norm);
/* Copy parameters and normalisation to host arrays (either may be NULL). */
dls_status dls_model_get(const dls_model* m, float* params, float* norm);
/* Outputs (n x 272, device) of raw features (n x 80, device, as written by
 * dls_features).  bf16 = 0: FP32 products; 1: bfloat16 operands, FP32
 * accumulation, the three layers in one fused kernel (the path encodes
 * use); 2: the same arithmetic layer by layer (bitwise equal to 1, kept as
 * its reference).  Other values: DLS_EINVAL. */
dls_status dls_model_forward(dls_model* m, const float* d_feat, int64_t n, int bf16, float* d_out,
                             void* stream);
/* Gradient (device, DLS_MODEL_NPARAM floats) and mean loss of one batch
 * without updating: d_rank (n, 1..16), d_basis (n x 256, target V[k][t]),
 * d_wb (n, window lengths).  *loss_out is written (host). */
dls_status dls_model_grad(dls_model* m, const float* d_feat, const int32_t* d_rank, const float* d_basis,
                          const int32_t* d_wb, int64_t n, int bf16, float* d_grad, float* loss_out,
                          void* stream);
/* One Adam step on one batch (same inputs as dls_model_grad). */
dls_status dls_model_train_step(dls_model* m, const float* d_feat, const int32_t* d_rank,
                                const float* d_basis, const int32_t* d_wb, int64_t n, float lr, int bf16,
                                float* loss_out, void* stream);
/* Raw features (nblocks x 80, device) of every block of the last dls_encode
 * on ctx, computed from d_field (the same field):  16 statistics (mean,
 * std, min, max, skewness, excess kurtosis, mean|dt|/std, std(dt)/std,
 * mean|dx|/std, mean|dy|/std, lag-1 and lag-2 temporal autocorrelation,
 * log10(mean x^2 / eps^2), log10(std / eps), time-mean energy fraction,
 * log2 M) then the 8 x 8 pooled time-mean image (normalised).  Blocks of
 * more than 256 points (which never take the warm start) get zeros.
 * field_bytes / out_bytes are the sizes of d_field and d_out in bytes.
 * DLS_EINVAL (nothing written) for windows above 16 steps, a field buffer
 * smaller than the last encode's field, or an output buffer smaller than
 * nblocks * 80 floats. */
dls_status dls_features(dls_ctx* ctx, const void* d_field, size_t field_bytes, float* d_out, size_t out_bytes,
                        void* stream);
/* Attach a model (NULL detaches), the number of subspace iterations
 * (0..64) and a rank margin (0..16: the warm start uses rhat + margin
 * columns, the acceptance test then keeps the smallest sufficient rank) for
 * encodes with DLS_LEARNED on this context. */
dls_status dls_ctx_set_model(dls_ctx* ctx, dls_model* m, int iters, int rank_margin);

/* Release a buffer returned by dls_finalize / dls_compress. */
void dls_free(void* p);

/* Thread-local description of the last error; valid until the next call. */
const char* dls_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* DLS_H */
