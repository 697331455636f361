/*
 * qkmps.h -- C ABI of the MI355X (gfx950) quantum-kernel MPS library.
 *
 * The library computes the quantum-kernel Gram matrix
 *     K[i][j] = |<psi(x_i) | psi(x_j)>|^2                      (Eq. (1))
 * where |psi(x)> = U(x)|+>^m is the paper's feature-map state (Eqs. (2)-(5)),
 * represented as a matrix product state (MPS, Sec. II-B) produced by truncated
 * MPS simulation of the circuit of Sec. II-C, and each overlap is contracted
 * site by site as in Fig. 2.
 *
 * Conventions shared by every entry point
 *   - Plain C types only; no C++ types or exceptions cross this boundary.
 *   - Every call returns a qk_status.  On failure a thread-local message is
 *     available from qk_last_error().  All argument checks happen before any
 *     device work is enqueued; a failed check enqueues nothing.
 *   - "dev" pointers are device (HBM) pointers owned by the caller.  "host"
 *     pointers are ordinary host memory owned by the caller.
 *   - Device work is asynchronous on the given HIP stream (a hipStream_t
 *     passed as void*; NULL = the default stream).  Host-returning calls
 *     (info, export, save) synchronise that stream first.
 *   - Batches (qk_mps_batch) are opaque and owned by the library; free them
 *     with mps_batch_free().  A batch lives on the device that was current
 *     when it was created.
 *   - Device faults surface as QK_EDEVICE at the next synchronising call.
 *
 * MPS storage (one batch = n MPS with the same qubit count m)
 *   Site l of MPS i is a complex tensor A[s][a][b], s in {0,1} the physical
 *   index, a < D_l and b < D_{l+1} the bond indices (D_0 = D_m = 1).  The
 *   batch stores every site with a padded shape [2][P_l][P_{l+1}], where the
 *   pad profile P_l is a multiple of 32 shared by the whole batch, and all
 *   padding is zero.  Exported MPS are left-canonical and normalised.
 */
#ifndef QKMPS_H
#define QKMPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QK_OK = 0,
  QK_EINVAL = -1,     /* invalid argument (NULL, size, NaN feature, mismatch) */
  QK_ENOMEM = -2,     /* device or host allocation failed                     */
  QK_EDEVICE = -3,    /* HIP runtime error or device fault                    */
  QK_ENOTSUP = -4,    /* valid but unsupported combination (e.g. chi > 128 in */
                      /* simulation, precision not packed)                     */
  QK_ENUMERIC = -5,   /* an SVD did not converge within its sweep limit       */
  QK_EABORTED = -6
} qk_status;

/* Arithmetic of the overlap contractions in mps_gram.  In every form the
 * final |overlap|^2 is formed in FP64. */
typedef enum {
  QK_FP64 = 0,        /* complex128 operands, FP64 MFMA                        */
  QK_FP32 = 1,        /* complex64 operands, FP32 MFMA, per-site 2^e rescale   */
  QK_SPLIT_BF16 = 2,  /* each real operand as a 31-bit fixed-point code with   */
                      /* one exponent per row / column, cut into four 8-bit    */
                      /* digits carried as bf16; the leading digit product     */
                      /* accumulates exactly in one FP32 MFMA accumulator, the */
                      /* smaller digit products of weight >= 2^-24 (and the   */
                      /* (2,2) product where bra ~ ket makes it one-signed)   */
                      /* in a second; FP64 combine                             */
  QK_SPLIT_I8 = 3     /* the same four digits as int8 MFMA operands; the ten  */
                      /* digit products of weight >= 2^-24 (and the (2,2)     */
                      /* product where bra ~ ket makes it one-signed)         */
                      /* accumulate exactly in int32, grouped by weight; FP64 */
                      /* combine                                              */
} qk_precision;

/* Circuit of Sec. II-C.  Rotation angles: Rz on qubit i uses coef_z * x_i;
 * Rxx on qubits (i, j) uses coef_xx * (1 - x_i) * (1 - x_j), with
 * Rz(t) = exp(-i t Z / 2) and Rxx(t) = exp(-i t XX / 2).  The paper's
 * bandwidth gamma corresponds to coef_z = 2 gamma, coef_xx = gamma^2 pi.  */
typedef struct {
  int32_t n_qubits;              /* m = features per point, >= 1             */
  int32_t interaction_distance;  /* d: edges (i, j) with 1 <= j - i <= d     */
  int32_t repetitions;           /* r of Eq. (3): Z layer then XX layer       */
  int32_t routing;               /* 0: 2(k-1) SWAPs around every Rxx at       */
                                 /*    distance k (Sec. II-C);                */
                                 /* 1: back-to-back inverse SWAPs of one      */
                                 /*    E_i block cancelled                    */
  double coef_z;
  double coef_xx;
  int32_t gate_split;            /* 1: apply each two-qubit gate through its  */
                                 /*    operator-Schmidt decomposition (the   */
                                 /*    gate SVD before application, footnote  */
                                 /*    of Sec. III-A): the kept count is at   */
                                 /*    most rank(G) x the bond between the    */
                                 /*    two sites, rank 2 for Rxx (1 at a zero */
                                 /*    angle), 4 for SWAP, so the gate's zero */
                                 /*    singular values never survive as       */
                                 /*    rounding noise; 0: plain theta SVD     */
  int32_t reserved[3];           /* must be zero                              */
} qk_circuit_spec;

/* Gate-list record: op 0 = RZ (site, feature), 1 = RXX (left site, feature i,
 * feature j), 2 = SWAP (left site).  Unused fields are -1. */
typedef struct {
  int32_t op, site, feat_i, feat_j;
} qk_gate;

typedef struct qk_mps_batch qk_mps_batch;

/* Per-batch simulation statistics. */
typedef struct {
  int64_t n;                 /* number of MPS                                  */
  int32_t m;                 /* sites                                          */
  int32_t max_bond;          /* largest bond dimension in the batch            */
  int32_t pad_max;           /* largest pad P_l                                */
  int32_t n_two_qubit_gates; /* per circuit (0 for imported batches)           */
  double max_discarded;      /* largest single-truncation discarded weight     */
  double mean_total_discarded; /* mean over MPS of the summed discarded weight */
  int64_t degenerate_cuts;   /* truncations whose kept/discarded gap < 1e-10   */
  int64_t unconverged_svds;  /* SVDs that hit the sweep limit                  */
  int64_t bytes_f64, bytes_f32, bytes_split_bf16; /* device bytes per form     */
  int64_t bytes_split_i8;
} qk_batch_info;

/* ---------------------------------------------------------------- setup */

/* Device-memory hook.  Every MPS is simulated once and its state reused by
 * many overlaps (Sec. II-D), so the batches that hold those states are long
 * lived and large; this hook lets them (and every scratch buffer the library
 * needs) live in the caller's memory pool, e.g. a framework's caching
 * allocator.
 *   alloc(bytes, ctx, stream): `bytes` of device memory on the current
 *       device, usable in stream order on `stream` (a hipStream_t as void*;
 *       NULL = the default stream), or NULL on failure (the library then
 *       returns QK_ENOMEM and enqueues nothing further for that call).
 *   free(ptr, ctx, stream): release a pointer returned by alloc; `stream` is
 *       the stream of its last use (NULL when it was last used in work the
 *       library has already synchronised).
 *   ctx: passed through unchanged.
 * Both function pointers must be non-NULL. */
typedef struct {
  void *(*alloc)(size_t bytes, void *ctx, void *stream);
  void (*free)(void *ptr, void *ctx, void *stream);
  void *ctx;
} qk_allocator;

/* Select HIP device `device` for subsequent calls on this thread and set the
 * allocator of that device: `alloc` (copied; its functions must stay valid
 * while the library uses them) or, with alloc == NULL, hipMalloc / hipFree
 * for batches and hipMallocAsync / hipFreeAsync for scratch.  The allocator
 * is registered before the device is selected, so it is in place even when
 * the call fails with QK_EDEVICE.  Batches keep the allocator that created
 * them and release their memory through it.  QK_EINVAL for a negative
 * device or an allocator with a NULL function. */
qk_status qk_init(int device, const qk_allocator *alloc);

/* Message of the last failed call on this thread ("" if none). */
const char *qk_last_error(void);

/* Library version string. */
const char *qk_version(void);

/* Gate list of a circuit spec (Sec. II-C; Eq. (3)).  Writes up to `cap`
 * records to `out_host` (may be NULL with cap 0) and the total count to
 * *n_gates.  QK_EINVAL if cap is too small (count still written). */
qk_status qk_circuit_compile(const qk_circuit_spec *spec, qk_gate *out_host,
                             int64_t cap, int64_t *n_gates);

/* ---------------------------------------------------------------- simulation */

/* Simulate |psi(x_i)> for every row of `features_dev` (n_points x n_qubits,
 * row-major FP64, any finite reals) with truncated MPS simulation
 * (Sec. II-B, Fig. 1): two-qubit gates are applied by contracting the gate
 * into the two site tensors, taking an FP64 SVD (batched one-sided Jacobi),
 * keeping k = max(1, min(chi_max, k_cut)) singular values, where k_cut is the
 * smallest count whose discarded weight sum_{i>=k} s_i^2 is at most
 * cutoff * sum_i s_i^2 (Eq. (8)); cutoff <= 0 disables weight truncation.
 * Kept values are renormalised to unit norm.  The orthogonality centre is
 * moved next to each gate before its SVD, and singular values are absorbed
 * toward the next two-qubit gate.  The result is left-canonical with the last
 * site normalised, stored in FP64; other precisions are packed on demand.
 * chi_max must be in [1, 128].  Above 64, two-site steps next to a bond
 * above 64 (Jacobi matrices up to 256 x 256) run with their matrices in a
 * scratch slot of 2 MiB per circuit of a launch (drawn from the device's
 * allocator for the call) and take tens of milliseconds each.  On success
 * *out receives a new batch. */
qk_status mps_simulate(const double *features_dev, int64_t n_points,
                       const qk_circuit_spec *spec, int32_t chi_max,
                       double cutoff, void *hip_stream, qk_mps_batch **out);

/* Progress callback: called on the calling thread with the number of
 * two-qubit gates applied so far and the total; a non-zero return value
 * aborts the simulation (QK_EABORTED, no batch returned). */
typedef int (*qk_progress_fn)(int64_t done, int64_t total, void *user);

/* mps_simulate with a progress callback invoked (after synchronising the
 * stream) every `every` two-qubit gates and once at the end.  `fn` may be
 * NULL, in which case this is mps_simulate. */
qk_status mps_simulate_progress(const double *features_dev, int64_t n_points,
                                const qk_circuit_spec *spec, int32_t chi_max,
                                double cutoff, void *hip_stream,
                                qk_progress_fn fn, void *user, int64_t every,
                                qk_mps_batch **out);

/* mps_simulate that also records how the MPS grows during the simulation
 * (the memory evolution of Sec. III-A, Fig. 6).  After the g-th two-qubit
 * gate of circuit i (g counted from 0 in circuit order, SWAPs included, as
 * in qk_circuit_compile without its Rz records), two int32 values are
 * written to trace_dev[(i * n2q + g) * 2 + {0, 1}]:
 *   [0] the bond dimension at the gate's cut (between its sites p, p+1);
 *   [1] sum_l D_l D_{l+1} over the MPS, i.e. its FP64 tensors take
 *       32 bytes times this value (2 physical values, 16-byte complex).
 * Both reflect every truncation and centre move up to that gate.
 * trace_dev is caller-owned device memory of n_points * n2q * 2 int32,
 * where n2q is the number of two-qubit gates of `spec`; it may be NULL only
 * if that product is 0 (QK_EINVAL otherwise).  The batch is bit-identical to
 * mps_simulate's. */
qk_status mps_simulate_trace(const double *features_dev, int64_t n_points,
                             const qk_circuit_spec *spec, int32_t chi_max,
                             double cutoff, int32_t *trace_dev,
                             void *hip_stream, qk_mps_batch **out);

/* mps_simulate with the simulation recorded once as a HIP graph and
 * replayed over the batch in chunks of circuits.  The graph holds every
 * launch that takes `circuits_per_graph` circuits from |+> through the whole
 * circuit to the normalised final state (Sec. II-B: gates, truncated SVDs,
 * centre moves); it is captured on a private stream, instantiated once and
 * launched ceil(n_points / circuits_per_graph) times, each replay on the
 * next chunk (the last one may be shorter), ordered after earlier work on
 * hip_stream and before later work on it.  0 picks equal chunks of at most
 * QK_GRAPH_CIRCUITS circuits.  Each circuit goes through the same steps with
 * the same kernels as in mps_simulate, so the batch is bit-identical; the
 * SVD scratch is sized for one chunk (512 KiB per circuit, plus 2 MiB for
 * chi_max above 64) instead of the whole batch, and the host launch work is that of one chunk whatever the
 * batch size.  QK_EINVAL if circuits_per_graph < 0; QK_EDEVICE if capture,
 * instantiation or a replay fails.  The call returns after the simulation
 * has finished. */
#define QK_GRAPH_CIRCUITS 1024
qk_status mps_simulate_graph(const double *features_dev, int64_t n_points,
                             const qk_circuit_spec *spec, int32_t chi_max,
                             double cutoff, int64_t circuits_per_graph,
                             void *hip_stream, qk_mps_batch **out);

/* ---------------------------------------------------------------- Gram */

/* Statistics of one Gram call (optional output of mps_gram*).  When a
 * stats pointer is given, the call waits for its launch to finish. */
typedef struct {
  int64_t entries;      /* overlaps contracted (a mirrored entry counts once) */
  int64_t tiles;        /* pair tiles in the work queue                       */
  int32_t workgroups;   /* persistent workgroups launched                     */
  int32_t tile_side;    /* pair-tile side of the kernel configuration         */
  int32_t queues;       /* work queues (1, or one per XCD)                    */
  int32_t block;        /* block size of the FP64 / FP32 forms (32, 64, 128)  */
  double flops;         /* algorithmic flops of the contracted overlaps: 8 per */
                        /* complex MAC of Fig. 2's site updates, counted from  */
                        /* the actual bond dimensions of every pair            */
  double kernel_ms;     /* duration of the Gram kernel (HIP events)           */
} qk_gram_stats;

/* K[i][j] = |<a_i | b_j>|^2 for i < na, j < nb, written to K_dev (row-major,
 * leading dimension ldk >= nb, FP64) following Fig. 2: for every site l,
 * E <- sum_s A_a[l][s]^H E A_b[l][s], starting from E = 1.
 * If b == NULL or b == a the matrix is symmetric: only i <= j is contracted
 * and mirrored (the diagonal is computed, not assumed).
 * `a` and `b` must have the same m.  The precision's packed form is built
 * (and kept) on first use.  The FP64 and FP32 forms support bond pads up
 * to 128 (bond dimensions up to 128; above 64 with E in a global scratch
 * slot of 2 x 128 x 128 complex values per workgroup, drawn from the
 * device's allocator for the call), the split forms up to 64: QK_ENOTSUP
 * for larger batches.  `stats` may be NULL. */
qk_status mps_gram(const qk_mps_batch *a, const qk_mps_batch *b,
                   qk_precision prec, double *K_dev, int64_t ldk,
                   void *hip_stream, qk_gram_stats *stats);

/* Block form for slabs and tile rows: rows a[a0 .. a0+na), columns
 * b[b0 .. b0+nb), written to K_dev[(i - a0) * ldk + (j - b0)].  With
 * upper_only != 0 (requires a == b) only entries with global j >= i are
 * contracted; each is also written to the transposed position (j, i) when
 * that position lies inside the block.  Other entries are left untouched. */
qk_status mps_gram_block(const qk_mps_batch *a, int64_t a0, int64_t na,
                         const qk_mps_batch *b, int64_t b0, int64_t nb,
                         int32_t upper_only, qk_precision prec,
                         double *K_dev, int64_t ldk, void *hip_stream,
                         qk_gram_stats *stats);

/* mps_gram_block for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, kernels and results as mps_gram_block (bit for bit, same
 * kernel configuration), without `stats`.  It allocates nothing: the work
 * queue (counters, job table and pair-tile list) lives in a static device
 * array of QK_NOALLOC_SCRATCH_BYTES per device, held from the library's
 * set-up on that device until the process ends, and both batches must
 * already hold the precision's packed planes (mps_batch_pack; QK_FP64 is
 * always present) and bond pads up to 64 (the kernels for pads up to 128
 * need per-workgroup scratch beyond the array) -- QK_ENOTSUP otherwise,
 * before any launch.  QK_EINVAL,
 * before any launch, when the work queue does not fit the array: with the
 * default pair tiles of side 16 that is about 520,000 tiles, e.g. a
 * symmetric Gram of up to ~16,000 MPS.  Every call on a device uses that
 * device's one array: calls that overlap in time on one device (other
 * threads, other streams) race and must be serialised by the caller. */
#define QK_NOALLOC_SCRATCH_BYTES (8u << 20)
qk_status mps_gram_block_noalloc(const qk_mps_batch *a, int64_t a0, int64_t na,
                                 const qk_mps_batch *b, int64_t b0, int64_t nb,
                                 int32_t upper_only, qk_precision prec,
                                 double *K_dev, int64_t ldk, void *hip_stream);

/* Several Gram jobs (different batches, qubit counts and pads) in ONE
 * persistent launch: workgroups pop tiles from a device work queue across
 * all jobs.  Each job is as in mps_gram_block with `upper_only` meaning
 * symmetric. */
typedef struct {
  const qk_mps_batch *a;
  const qk_mps_batch *b;   /* == a with upper_only != 0 for symmetric jobs */
  int64_t a0, na, b0, nb;
  int32_t upper_only;
  int32_t reserved;
  double *K_dev;
  int64_t ldk;
} qk_gram_job;

qk_status mps_gram_multi(const qk_gram_job *jobs, int32_t n_jobs,
                         qk_precision prec, void *hip_stream,
                         qk_gram_stats *stats);

/* Autotuner of the Gram kernels' tile shapes.  For `prec` and the bond-pad
 * bucket of batch `b` (pads <= 32, <= 64 or <= 128), every valid configuration
 * (block size 32 or 64 for the FP64 / FP32 forms when the pads allow, 128
 * above 64, pair-tile
 * side 8 / 16 / 32, one work queue or one per XCD) computes the symmetric
 * Gram of the first min(sample, n) MPS of `b` (one warm-up run, then the
 * best of two timed runs, wall clock including the launch's host work).
 * The fastest configuration, if it beats the default by more than 2 % (the
 * timing's run-to-run spread is about 1 %), else the default, is stored for
 * this device, precision and pad bucket and used by every later mps_gram*
 * call on this process; `report` (may be NULL) receives it with its time and
 * the default configuration's time.  Not thread-safe with concurrent Gram calls of the same bucket. */
typedef struct {
  int32_t maxp;           /* block size of the winning configuration        */
  int32_t tile_side;      /* pair-tile side                                  */
  int32_t queues;         /* 1 or one per XCD                                */
  int32_t n_candidates;   /* configurations timed                            */
  double best_ms;         /* wall time of the winner on the sample           */
  double default_ms;      /* wall time of the default configuration          */
} qk_tune_report;

qk_status mps_gram_autotune(qk_mps_batch *b, qk_precision prec, int64_t sample,
                            void *hip_stream, qk_tune_report *report);

/* Forget every stored configuration (back to the defaults). */
qk_status mps_gram_tune_reset(void);

/* ---------------------------------------------------------------- batches */

/* Build an MPS batch from host FP64 tensors.  `dims_host` holds n x (m+1)
 * bond dimensions (first and last 1).  `tensors_host` holds, for MPS 0..n-1
 * and site 0..m-1 in order, the complex tensor A[s][a][b] with s in {0,1},
 * a < D_l, b < D_{l+1}, as interleaved (re, im) doubles, densely packed.
 * Bond dimensions must be in [1, 128]. */
qk_status mps_batch_import(const double *tensors_host, const int32_t *dims_host,
                           int64_t n, int32_t m, void *hip_stream,
                           qk_mps_batch **out);

qk_status mps_batch_info(const qk_mps_batch *b, qk_batch_info *info);

/* n x (m+1) bond dimensions into host memory. */
qk_status mps_batch_bond_dims(const qk_mps_batch *b, int32_t *dims_host);

/* Per-MPS statistics into host arrays of length n (any may be NULL):
 * summed discarded weight, number of near-degenerate cuts. */
qk_status mps_batch_trunc_stats(const qk_mps_batch *b, double *discarded_host,
                                int32_t *degenerate_host);

/* FP64 tensors of MPS `idx` in the densely packed import layout.  `cap` is
 * the capacity in doubles; QK_EINVAL if too small.  *written = doubles used. */
qk_status mps_batch_export(const qk_mps_batch *b, int64_t idx, double *host_buf,
                           int64_t cap, int64_t *written);

/* Build the packed operand planes of `prec` now (otherwise built by the first
 * mps_gram with that precision).  QK_FP64 is always present. */
qk_status mps_batch_pack(qk_mps_batch *b, qk_precision prec, void *hip_stream);

/* Release the packed planes of `prec` (not QK_FP64). */
qk_status mps_batch_drop(qk_mps_batch *b, qk_precision prec);

/* Forms selected in mps_batch_gather. */
#define QK_FORM_FP64 1u
#define QK_FORM_FP32 2u
#define QK_FORM_SPLIT_BF16 4u
#define QK_FORM_SPLIT_I8 8u

/* New batch holding copies of MPS idx[0..count) of `src` (indices may
 * repeat), in the forms selected by `forms` (QK_FORM_* bits; each must be
 * present in `src`).  A batch without the FP64 form can only be used by
 * mps_gram in the forms it holds (export and packing return QK_ENOTSUP). */
qk_status mps_batch_gather(const qk_mps_batch *src, const int64_t *idx_host,
                           int64_t count, uint32_t forms, void *hip_stream,
                           qk_mps_batch **out);

/* Keep a batch across runs: every MPS is simulated once and its state
 * reused (Sec. II-D), so a simulated training set can be written to a file
 * and loaded later instead of simulated again.
 * mps_batch_save writes, little-endian:
 *   "QKMPSB01" (8 bytes); int32 m; int32 n_two_qubit_gates; int64 n;
 *   int32 pad[m + 1]; int32 dims[n][m + 1];
 *   double summed_discarded[n]; double max_discarded[n];
 *   int32 degenerate_cuts[n]; int32 unconverged_svds[n];
 *   the FP64 tensors, MPS after MPS, site after site, each site the padded
 *   complex block [s][P_l][P_{l+1}] as interleaved (re, im) doubles (zero
 *   beyond the bond dimensions).
 * The batch must hold the FP64 form (QK_ENOTSUP otherwise).  The call
 * synchronises the device.  QK_EINVAL for a NULL argument or a file that
 * cannot be written (the message says why). */
qk_status mps_batch_save(const qk_mps_batch *b, const char *path);

/* Read a file written by mps_batch_save into a new batch on the current
 * device (allocated through the registered allocator); packed forms are
 * built on demand as after mps_simulate.  QK_EINVAL for a missing,
 * truncated or malformed file (bad magic, sizes that do not match the
 * header, a bond dimension outside [1, 128] or above its pad, a pad that is
 * not a multiple of 32, a non-finite tensor entry).  On success *out
 * receives the batch; the call returns after the data are on the device. */
qk_status mps_batch_load(const char *path, void *hip_stream, qk_mps_batch **out);

void mps_batch_free(qk_mps_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* QKMPS_H */
