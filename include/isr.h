/*
 * isr.h -- in-situ snapshot reduction on MI355X (gfx950): the C ABI.
 *
 * The operation (arXiv 2407.20731, Sec. IV-B, "Turbulence with data
 * compression"): while a spectral-element (SEM) velocity snapshot is still in
 * GPU memory, reduce it with the physics-based, JPEG-inspired lossy step --
 * keep only the Legendre coefficients of the most energetic motions and drop
 * the rest under a maximal allowed error.  Per velocity component the library
 *
 *   1. transforms every hexahedral element's GLL nodal values u[k][j][i] to
 *      Legendre coefficients c[r][q][p] (tensor product of A = V^-1, with
 *      V[i][k] = P_k(xi_i) at the Gauss-Lobatto-Legendre nodes xi),
 *   2. forms the GLL mass-weighted norm U2 = sum_e sum_kji (J_e w_k w_j w_i) u^2
 *      and the coefficient energies e = (J_e g_r g_q g_p) c^2 (g = discrete
 *      GLL norms of the Legendre polynomials: 2/(2k+1), and 2/N for k = N),
 *   3. finds the global value threshold tau, the largest energy value such
 *      that the dropped energy S(tau) = RN(exact sum of energies < tau) does
 *      not exceed B = (tol*tol)*U2 (FP64, exact sums, no sort),
 *   4. compacts the kept coefficients (e >= tau) into a blob: a bitmap, a
 *      per-element offset table and the kept values,
 *   5. inverse-transforms the kept set and measures the relative
 *      mass-weighted L2 error sqrt(err2/U2); if rounding pushed it above tol,
 *      it lowers B by (tol/rel)^2 * (1 - 2^-20) and repeats 3-5 (at most 4
 *      times; then ISR_ETOL).
 *
 * With ISR_PREC_FP64, U2, S and err2 are the correctly rounded values of the
 * exact sums of their FP64 terms, and the transforms use one fixed
 * evaluation order (see isr_forward), so every coefficient, energy and
 * threshold is reproducible bit for bit by a CPU implementation of the same
 * definition.  With ISR_PREC_FP32 / ISR_PREC_BF16, whose energies and
 * reconstruction carry the transform error anyway, each lane adds its norm,
 * energy and error terms in a fixed FP64 order and only the lane totals are
 * combined exactly: U2, S and err2 are deterministic (the same alone, in a
 * batch or in the serving mix) but not correctly rounded: the relative error
 * is at most (terms per lane) 2^-53, which stays below 1e-12 up to about 10^6
 * elements at N = 7 (the typical error is far smaller).
 * On these paths U2 still comes from the FP64 field and FP64 products.
 *
 * Conventions
 *   - Every function returns an int status (ISR_OK or a negative ISR_E*),
 *     except isr_last_error and isr_blob_free.  On error, output handles are
 *     set to NULL and isr_last_error() describes the failure.
 *   - "device pointer" = memory on the context's GPU (hipMalloc, or a torch
 *     CUDA tensor's data_ptr()).  The library never frees caller memory.
 *   - Streams are hipStream_t passed as void*; NULL = the default stream.
 *   - A context serialises its own calls and may be used from several host
 *     threads.  No C++ exception crosses this ABI.
 */
#ifndef ISR_H
#define ISR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define ISR_OK 0
#define ISR_PENDING 1       /* isr_poll: request not finished yet */
#define ISR_EINVAL (-1)     /* bad argument (see each call) or non-finite field */
#define ISR_ENOMEM (-2)     /* footprint above the HBM budget, or allocation failed */
#define ISR_EDEVICE (-3)    /* a HIP call failed */
#define ISR_ETOL (-4)       /* error bound not met after the rounding repair */
/* (-5 is not used) */
#define ISR_ENOTFOUND (-6)  /* unknown request id */

/* ---- precisions of the transforms ------------------------------------- */
#define ISR_PREC_FP64 0   /* VALU FP64, fixed order, no FMA: bit-exact */
#define ISR_PREC_FP32 1   /* FP32 MFMA, FP32 accumulation; FP64 norms/select */
#define ISR_PREC_BF16 2   /* BF16 MFMA (split operands), FP32 accumulation */

/* ---- context flags ---------------------------------------------------- */
#define ISR_FLAG_TIMING 1u  /* record device time per phase into isr_stats */
#define ISR_FLAG_BATCH_PERSISTENT 4u /* FP32/BF16 batches of 8 snapshots or more, orders 5/7/9: one
                                        persistent launch of the streaming path instead of one
                                        streaming pipeline per snapshot on the scheduler's streams */

#define ISR_MAX_COMP 8
#define ISR_MAX_ORDER 15
#define ISR_NPHASE 9

typedef struct isr_ctx isr_ctx;
typedef struct isr_blob isr_blob;

typedef struct {
  int32_t device;            /* HIP device ordinal */
  uint32_t flags;            /* ISR_FLAG_* */
  uint64_t hbm_budget_bytes; /* cap on device memory the library holds; 0 = 64 GiB */
  int32_t max_inflight;      /* isr_submit: requests resident at once; 0 = 8 */
  int32_t host_threads;      /* isr_pack_submit: host threads of the lossless
                                stage; 0 = 12 (or the host's cores, if fewer) */
  const char *autotune_path; /* optional tile-shape table: read at create when
                                present, written by isr_autotune; NULL = none */
} isr_config;

/* One snapshot to compress.
 *   field        DEVICE pointer, FP64.  Component c, element e, node (k, j, i)
 *                is field[c * comp_stride + e * n^3 + (k * n + j) * n + i],
 *                n = order + 1 (element-local SEM storage, i fastest, shared
 *                face nodes duplicated).  Must be 8-byte aligned (16-byte
 *                aligned tiles are read with 16-byte loads).  Borrowed:
 *                it must stay unchanged until isr_compress returns or
 *                isr_poll reports completion.  All values must be finite.
 *   n_elem       number of elements, >= 1, and n_elem * n^3 < 2^32.
 *   order        polynomial order N in [1, ISR_MAX_ORDER].
 *   ncomp        velocity components in [1, ISR_MAX_COMP]; each gets its own
 *                threshold (per-component relative bound).
 *   comp_stride  values between components; 0 means n_elem * n^3.
 *   tol          relative mass-weighted L2 bound per component, >= 0; a
 *                negative tol keeps every coefficient (lossless transform).
 *   precision    ISR_PREC_*.
 *   flags        0, or ISR_FIELD_COPY (isr_submit only): copy-on-submit.
 *                isr_submit copies the field (and elem_jac) into the
 *                library's HBM arena on `stream` before it returns, so the
 *                caller may overwrite them with work enqueued on `stream`
 *                right away (from the host or another stream: after
 *                synchronising with `stream`).  The copy counts against the
 *                HBM budget until the request completes; when the budget
 *                cannot hold it at submit time, isr_submit returns
 *                ISR_ENOMEM.  Without the flag the field is borrowed.
 *   elem_jac     optional DEVICE pointer to n_elem positive FP64 Jacobians of
 *                affine elements (constant per element); NULL means 1.
 *   stream       hipStream_t on which `field` was produced; the library's
 *                work is ordered after it.
 */
#define ISR_FIELD_COPY 1
typedef struct {
  const double *field;
  int64_t n_elem;
  int32_t order;
  int32_t ncomp;
  int64_t comp_stride;
  double tol;
  int32_t precision;
  int32_t flags;
  const double *elem_jac;
  void *stream;
} isr_field;

/* Per-result statistics (arrays are per component). */
typedef struct {
  double norm2[ISR_MAX_COMP];    /* U2 */
  double budget[ISR_MAX_COMP];   /* B actually used (after any repair) */
  double tau[ISR_MAX_COMP];      /* threshold; +inf = nothing kept; 0 = all kept */
  double dropped[ISR_MAX_COMP];  /* S(tau) */
  double err2[ISR_MAX_COMP];     /* measured mass-weighted squared error */
  double rel_err[ISR_MAX_COMP];  /* sqrt(err2 / U2), 0 when U2 == 0 */
  uint64_t kept[ISR_MAX_COMP];
  uint64_t in_bytes;             /* ncomp * n_elem * n^3 * 8 */
  uint64_t blob_bytes;           /* serialized blob size */
  double cr;                     /* (in_bytes - blob_bytes) / in_bytes */
  double t_submit, t_start, t_done; /* host monotonic seconds */
  float phase_ms[ISR_NPHASE];    /* ISR_FLAG_TIMING: device ms per phase:
                                    0 norm+histogram pass, 1 threshold select,
                                    2 candidate pass, 3 refine, 4 compact+verify
                                    pass, 5 finalize, 6 repair total, 7 an
                                    abandoned streaming attempt (see path),
                                    8 zero fill and sampling pass with its
                                    window selection (ahead of phase 0) */
  int32_t repair_iters;
  int32_t status;
  int32_t precision;
  int32_t path;                  /* 1: streaming path (threshold inside the
                                    sampled window); 2: the same, inside the
                                    persistent batch launch; 0: general
                                    pipeline (orders without a streaming path,
                                    or the window missed and the request was
                                    rerun) */
} isr_stats;

/* Create a context on cfg->device (cfg may be NULL: device 0, defaults).
 * Computes the GLL/Legendre tables on the host for every order and uploads
 * them (the element basis of the lossy step, Sec. IV-B).  Errors:
 * ISR_EINVAL, ISR_EDEVICE. */
int isr_create(const isr_config *cfg, isr_ctx **out);

/* Destroy a context: waits for its requests, frees its device memory.  Blobs
 * of this context must be freed first.  (Runtime only: no passage of the
 * paper defines it.) */
int isr_destroy(isr_ctx *ctx);

/* Text of the last error on the calling thread (valid until its next call). */
const char *isr_last_error(void);

/* Compress one snapshot and wait for the result: steps 1-5 above, the lossy
 * step of Sec. IV-B run synchronously on the application's GPU (the
 * synchronous approach of Sec. III-A).  On ISR_OK or ISR_ETOL,
 * *out receives a device-resident blob owned by the caller (isr_blob_free);
 * with ISR_ETOL the blob's measured error exceeds tol.  st may be NULL.
 * Errors: ISR_EINVAL (null/misaligned pointer, order, n_elem, ncomp, NaN
 * tol, bad precision, non-finite field values), ISR_ENOMEM, ISR_EDEVICE. */
int isr_compress(isr_ctx *ctx, const isr_field *f, isr_blob **out, isr_stats *st);

/* ---- allocation-free compression ----------------------------------------
 * (Runtime only: no passage of the paper defines it.)
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * compression as isr_compress (same kernels, same result, byte for byte),
 * but the call allocates nothing: no hipMalloc / hipFree, no host or pinned
 * allocation.  Its scratch is a fixed device array of the library,
 * ISR_NOALLOC_SCRATCH_BYTES per GPU, held by every GPU the library runs on
 * until the process ends; a request whose scratch exceeds it is refused with
 * ISR_ENOMEM (about 20 bytes per value plus 2.1 MB: at N = 7 with 3
 * components, up to about 4,200 elements).  The blob is written to the caller's
 * buffer.
 *   d_out      DEVICE pointer, 256-byte aligned, out_cap bytes; receives the
 *              serialized blob (the bytes isr_blob_to_host would give, layout
 *              below).  out_cap must hold the worst case (every coefficient
 *              kept): 64 + 72 ncomp + 8 ncomp n_elem W + 8 ncomp (n_elem + 1)
 *              + ncomp n_elem n^3 value_bytes; otherwise ISR_EINVAL.
 *   out_bytes  receives the blob's size (on ISR_EINVAL for a short buffer:
 *              the size required).  May be NULL.
 * Blocking: returns once the blob and *st are complete.  Returns ISR_OK or
 * ISR_ETOL (the blob is written in both cases), else an error as
 * isr_compress.  Every call on one GPU uses the same scratch array, which
 * keeps the last call's contents (the pipeline clears what must start at
 * zero); the library runs these calls one at a time per GPU, since calls
 * that overlapped on one GPU would race on it. */
#define ISR_NOALLOC_SCRATCH_BYTES (128ull << 20)
int isr_compress_noalloc(isr_ctx *ctx, const isr_field *f, void *d_out, uint64_t out_cap, uint64_t *out_bytes,
                         isr_stats *st);

/* Quantised variant of the lossy step (the JPEG-like form: the kept
 * coefficients are quantised, as JPEG quantises the coefficients it keeps).
 * FP64 path, unit Jacobians (f->elem_jac NULL), f->tol >= 0, 0 <= share < 1.
 * Per component: the plain method's global cut at the budget
 * ((tol*tol)*U2)*(1 - share) (dropped energy S_c, K kept), then each kept
 * coefficient c (flat index f) coded as q = rint((c sqrt(g3_f)) / step) with
 * step = (2 sqrt((B - S_c) / K)) (1 - 2^-20), B = (tol*tol)*U2, so that every
 * code's error energy is at most (step/2)^2 and the total stays below B; the
 * exact error of the dequantised field (values (q step) / sqrt(g3_f), FP64
 * fixed-order inverse, the one isr_decompress uses) is measured, and the step
 * is shrunk by (tol/rel)(1 - 2^-20) while rounding leaves it above tol (at
 * most 4 times; then ISR_ETOL).  The blob holds the codes as FP32 integers
 * (value kind 1) and the step per component; isr_decompress dequantises.
 * Errors: as isr_compress; ISR_EINVAL for another precision, Jacobians, a
 * negative tol or share outside [0, 1); ISR_ETOL when a code would need more
 * than 24 bits. */
int isr_compress_quantized(isr_ctx *ctx, const isr_field *f, double share, isr_blob **out, isr_stats *st);

/* Per-element cut, a variant of the selection (Sec. IV-B: the lossy step's
 * sorting kernels, read as a selection made element by element).  FP64
 * path, f->tol >= 0, Jacobians allowed, n_elem < 2^32.  Every element e of a
 * component is cut alone by the plain value rule: U2_e = RN(exact sum of its
 * norm terms), budget B_e = ((tol*tol)*U2_e)*s, threshold tau_e = the largest
 * of its energies v (or +inf) with RN(exact sum of its energies below v) <= B_e;
 * kept = energies >= tau_e.  U2, err2 and the dropped energy are the exact
 * component totals as in isr_compress, B = (tol*tol)*U2, and the blob's tau
 * is NaN (the thresholds are per element).  While rounding leaves rel above
 * tol, s <- (s*((tol/rel)*(tol/rel)))*(1 - 2^-20), at most 4 times; then
 * ISR_ETOL.  Each element then keeps its own relative error within tol, up
 * to rounding, at the price of more kept coefficients than the global cut.
 * The blob has the layout of isr_compress's FP64 blobs.  Errors: as
 * isr_compress; ISR_EINVAL for another precision or a negative tol. */
int isr_compress_elemcut(isr_ctx *ctx, const isr_field *f, isr_blob **out, isr_stats *st);

/* Compress several snapshots (orders may differ) in one batched launch
 * sequence (the lossy step of Sec. IV-B over the snapshots a run writes
 * periodically, several of them at once).  FP64 snapshots of orders 5, 7 and 9: one persistent launch of
 * the general passes.  FP32 / BF16: one streaming pipeline per snapshot on
 * the scheduler's streams, largest first; with ISR_FLAG_BATCH_PERSISTENT and
 * at least 8 snapshots of orders 5, 7 and 9, one persistent launch of the
 * streaming path, each snapshot with the tile shape the context holds for
 * its order and precision (built-in, or set by isr_autotune / isr_set_tile;
 * the kernel holds every candidate shape).  Other batches: one pipeline per
 * snapshot.  Results are the same in every form.  outs[i] / st[i] as in isr_compress; returns the first non-OK
 * status (each st[i].status holds its own).  Footprint of the whole batch must
 * fit the budget (ISR_ENOMEM otherwise). */
int isr_compress_batch(isr_ctx *ctx, const isr_field *fs, int32_t count, isr_blob **outs,
                       isr_stats *st);

/* Queue a snapshot for compression and return at once with a request id
 * (the application continues while the lossy step runs: the asynchronous
 * side of Sec. III-A's hybrid approach).
 * Requests are admitted to the device while their footprint fits the HBM
 * budget and fewer than max_inflight are resident; later arrivals join the
 * running ones (continuous batching).  The field must stay unchanged until
 * isr_poll reports completion, unless f->flags holds ISR_FIELD_COPY
 * (copy-on-submit, above).  Errors as isr_compress (argument checks only;
 * ISR_ENOMEM if the request alone exceeds the budget, or its copy does not
 * fit it now). */
int isr_submit(isr_ctx *ctx, const isr_field *f, uint64_t *req);

/* Poll a request: ISR_PENDING while running; otherwise the request's final
 * status (ISR_OK, ISR_ETOL, or an error) with *out / *st filled, and the
 * request id is retired.  wait_ms > 0 blocks up to that long; < 0 blocks
 * until done.  ISR_ENOTFOUND for an unknown or retired id. */
int isr_poll(isr_ctx *ctx, uint64_t req, int32_t wait_ms, isr_blob **out, isr_stats *st);

/* Reconstruct the nodal field from a blob (Sec. IV-B: the kept coefficients
 * transformed back; the error bound is stated on this field) into d_out
 * (DEVICE, same layout as
 * the input with comp_stride = n_elem * n^3), FP64 (out_prec ISR_PREC_FP64)
 * or FP32 (ISR_PREC_FP32).  The inverse is the one whose result the
 * compression measured, so the blob's rel_err is the error of this output:
 * FP64 blobs use the FP64 inverse in the fixed order (that of isr_forward,
 * with V); FP32 / BF16 blobs repeat, bit for bit, the MFMA inverse of the
 * engine that compressed them (recorded in the blob).  Enqueued on `stream`;
 * the call returns after enqueueing.  Errors: ISR_EINVAL, ISR_EDEVICE. */
int isr_decompress(isr_ctx *ctx, const isr_blob *b, void *d_out, int32_t out_prec, void *stream);

/* Forward transform only (step 1 above, Sec. IV-B; no truncation):
 * coefficients c[comp][e][r][q][p] (p fastest) into d_coef (DEVICE, FP64 for ISR_PREC_FP64, else FP32), in
 * the requested precision.  FP64 order: t1 = sum_i A[p][i] u[k][j][i], then
 * t2 = sum_j A[q][j] t1[k][j][p], then c = sum_k A[r][k] t2[k][q][p], each
 * sum started from its first product and accumulated in ascending index with
 * separately rounded multiply and add.  Synchronous. */
int isr_forward(isr_ctx *ctx, const isr_field *f, void *d_coef);

/* Blob queries and (de)serialisation of the compressed snapshot (Sec. IV-B:
 * the kept coefficients and where they sit; its size gives the compression
 * ratio of Sec. IV-C).  Serialized layout (little endian):
 *   "ISR1", u32 version=3, i32 order, i32 ncomp, i64 n_elem, i32 value_bytes
 *   (8 or 4), i32 words_per_elem W = ceil(n^3/64), f64 tol, i32 precision,
 *   i32 status, i32 engine (FP32 / BF16: 0 general passes, 1 wave-tile or
 *   large-order engine, 2 dense-tile engine; 0 for FP64), i32 tile (the
 *   dense tile, else 0), i32 value kind (0 coefficient values, 1
 *   quantisation codes: integers held exactly by FP32, isr_compress_quantized),
 *   i32 0; then per component: f64 U2, B, tau, dropped, err2, rel_err,
 *   u64 kept, u64 values_offset, f64 quantisation step (0 unless value kind
 *   1); then all bitmaps [ncomp][n_elem][W] u64 (bit
 *   f = p + n q + n^2 r of element e set iff kept), all offset tables
 *   [ncomp][n_elem + 1] u64 (per component, starting at 0), all kept values
 *   (component after component, element then f ascending). */
int isr_blob_info(const isr_blob *b, int32_t *order, int32_t *ncomp, int64_t *n_elem,
                  int32_t *value_bytes);
int isr_blob_size(const isr_blob *b, uint64_t *bytes);
int isr_blob_to_host(const isr_blob *b, void *buf, uint64_t cap);
int isr_blob_from_host(isr_ctx *ctx, const void *buf, uint64_t n, isr_blob **out);
void isr_blob_free(isr_blob *b);

/* ---- hybrid lossless stage (host CPU cores) ------------------------------
 * The paper's hybrid approach (arXiv 2407.20731, Sec. III-A, IV-B): the lossy
 * step runs synchronously on the GPU, and its output is then coded
 * losslessly on separate host cores, asynchronously, while the GPU goes on.
 * Packed format (little endian): "ISRZ", u32 version = 1, u32 codec, u32
 * flags, u64 raw bytes, u32 chunk count K, u32 raw bytes per chunk, K x u64
 * coded chunk sizes, then the K independently coded chunks of the raw
 * stream.  The raw stream is the serialized blob; with ISR_PACK_SHUFFLE its
 * kept values are stored byte plane by byte plane.  Compression ratio of the
 * whole chain: (input bytes - packed bytes) / input bytes (Sec. IV-C). */
#define ISR_CODEC_ZLIB 1   /* deflate (zlib), levels 0-9 */
#define ISR_CODEC_BZIP2 2  /* bzip2, block sizes 1-9 (x 100 kB) */
#define ISR_PACK_SHUFFLE 1u

/* Host-only: code a serialized blob (isr_blob_to_host bytes) with `threads`
 * host threads (0 = 12 or the host's cores).  out == NULL: only *out_bytes
 * (the packed size).  Errors: ISR_EINVAL (bad codec, level, flags or blob,
 * short buffer). */
int isr_pack_host(const void *blob, uint64_t n, int32_t codec, int32_t level, uint32_t flags, int32_t threads,
                  void *out, uint64_t cap, uint64_t *out_bytes);

/* Host-only: decode a packed blob back to the serialized blob (out == NULL:
 * only its size in *out_bytes).  Errors: ISR_EINVAL (corrupt input, short
 * buffer). */
int isr_unpack_host(const void *packed, uint64_t n, void *out, uint64_t cap, uint64_t *out_bytes);

/* Queue a device blob for lossless coding on the context's host threads:
 * its bytes are copied to pinned host memory on the packer's own stream
 * (asynchronous to the caller's and the compression streams) and coded in
 * submission order.  The blob must stay unfreed until the job completes.
 * Errors: ISR_EINVAL, ISR_ENOMEM (pinned staging), ISR_EDEVICE. */
int isr_pack_submit(isr_ctx *ctx, const isr_blob *b, int32_t codec, int32_t level, uint32_t flags, uint64_t *job);

/* Poll a packing job: ISR_PENDING while it runs (wait_ms as isr_poll); then
 * *out_bytes = packed size and *seconds = submit-to-done time.  With out ==
 * NULL the job stays (size query); with a buffer of cap >= the size the bytes
 * are copied and the job is retired.  Errors: ISR_ENOTFOUND, ISR_EINVAL. */
int isr_pack_poll(isr_ctx *ctx, uint64_t job, int32_t wait_ms, void *out, uint64_t cap, uint64_t *out_bytes,
                  double *seconds);

/* ---- tile shapes and the autotuner --------------------------------------
 * (Runtime only: no passage of the paper defines them.)  The FP32 / BF16 streaming passes come in several tile shapes per order.
 * Shape 0 is the wave-tile engine: a wavefront owns 64 / (N+1)^2 elements
 * (one from N = 7 up) and works in the MFMA register layout.  Shape T > 0 is
 * the dense-tile engine: a wavefront owns T consecutive elements and does all
 * per-value work (norm, energies, window tests, keep decisions, bitmaps,
 * ranks, error terms) in dense order.  Every shape meets the same bound and
 * passes the same checks, and one shape always gives the same result; but
 * the FP32 / BF16 energy and error sums add each lane's terms in that lane's
 * order, so two shapes can differ in the last bits of S and err2 (and then in
 * coefficients at the threshold).
 * The table starts
 * from the built-in choice, or from config.autotune_path when that file
 * exists (text lines "order precision tile"). */
typedef struct {
  int32_t count;     /* candidates timed */
  int32_t tile[16];  /* their shapes */
  double ms[16];     /* best wall-clock milliseconds of one compression each */
  int32_t best;      /* shape now in the table */
} isr_tune_report;

/* Shape in use for (order, precision).  Errors: ISR_EINVAL. */
int isr_get_tile(isr_ctx *ctx, int32_t order, int32_t precision, int32_t *tile);

/* Use shape `tile` for (order, precision) from the next request on: a
 * compiled shape, 0, or -1 for the built-in choice.  Requests already
 * admitted keep theirs.  Errors: ISR_EINVAL (FP64, an order without a
 * streaming path, a shape that is not compiled). */
int isr_set_tile(isr_ctx *ctx, int32_t order, int32_t precision, int32_t tile);

/* Autotuner: compress f with every candidate shape of (f->order,
 * f->precision), one warm-up call and then the best of `reps` timed calls
 * each, keep the fastest in the table and, when config.autotune_path was
 * given, rewrite that file with the whole table.  f should look like the
 * production snapshots (its size matters).  Requests of the same (order,
 * precision) submitted meanwhile may run with a candidate shape.  rep may be
 * NULL.  Errors: as isr_compress; ISR_EINVAL for FP64 (it has one shape). */
int isr_autotune(isr_ctx *ctx, const isr_field *f, int32_t reps, isr_tune_report *rep);

/* Host-only: the library's own FP64 tables for order N, the GLL basis of the
 * lossy step (Sec. IV-B); each entry is the correctly rounded value of the
 * exact quantity: xi[n], w[n], V[n*n]
 * (V[i*n+k] = P_k(xi_i)), A[n*n] (A[p*n+i] = (V^-1)[p][i]), gamma[n],
 * w3[n^3] (w3[(k*n+j)*n+i] = w_k w_j w_i), g3[n^3] (gamma_r gamma_q gamma_p).
 * Any pointer may be NULL.  No GPU needed.  Errors: ISR_EINVAL. */
int isr_gll_tables(int32_t order, double *xi, double *w, double *V, double *A, double *gamma,
                   double *w3, double *g3);

/* Library version string. */
const char *isr_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ISR_H */
