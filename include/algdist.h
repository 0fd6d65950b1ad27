/*
 * algdist.h -- C ABI of libalgdist.so, the MI355X (gfx950) implementation of
 * the data-parallel hot path of algebraic-distance AMG setup:
 *
 *   1. relax K test vectors on A x = 0            (setup_testvectors)
 *   2. per-edge least-squares algebraic distance  (algebraic_distance)
 *   3. strength graph from the distances          (strength_graph)
 *   4. least-squares interpolation rows           (ls_interp)
 *
 * after Brandt, Brannick, Kahl, Livshits, "An algebraic distances measure of
 * AMG strength of connection" (arXiv:1106.5990).  Section and equation names
 * below are that paper's.
 *
 * Conventions for every call
 * --------------------------
 * - All array arguments are DEVICE pointers unless marked "host".  The caller
 *   allocates and owns every buffer; the library never frees caller memory.
 *   The handle owns only its internal workspace (grown on demand, freed by
 *   algdist_destroy).
 * - Every compute call is asynchronous on `stream` (a hipStream_t passed as
 *   void*; NULL = the legacy default stream) and returns after enqueueing.
 * - Return value: an ad_status.  Argument errors are detected on the host,
 *   before anything is enqueued, and leave all outputs untouched; the
 *   message is available from algdist_last_error().  Conditions that can only
 *   be seen on the device (a zero diagonal, a bad colour, a non-finite
 *   distance, a malformed CSR in csr_validate) set bits of a sticky device
 *   status word read by algdist_status().
 * - CSR: int32 row_ptr[n+1] (row_ptr[0] = 0, nondecreasing), int32 col[nnz]
 *   sorted ascending within each row with the diagonal present, values of
 *   the type named by `dtype`.  Panels (test vectors) are row-major n x K:
 *   entry (i, k) at X[i*K + k], K contiguous; the panel type is the CSR's
 *   dtype.  Device pointers to panels must be 16-byte aligned.
 * - K must be one of 2, 4, 8, 16, 32, 64.
 * - Calls on one handle must not overlap in time across host threads.
 * - Graph capture: a call may be made while `stream` is capturing (its
 *   launches are then recorded into the caller's graph).  Workspace and
 *   batch tables do not move under such a graph: a call that would have to
 *   grow the workspace, or upload batch tables for a new argument set,
 *   during capture returns AD_EUNSUPPORTED (make the same call once
 *   uncaptured first); buffers a captured graph refers to are kept alive
 *   until algdist_destroy, even when a later uncaptured call needs larger
 *   ones.  Replays and other calls on the handle share its workspace as
 *   scratch, so they must not overlap in time either.
 */
#ifndef ALGDIST_H
#define ALGDIST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ALGDIST_VERSION 1

typedef enum { AD_F32 = 0, AD_F64 = 1 } ad_dtype;
typedef enum { AD_JACOBI = 0, AD_MULTICOLOR_GS = 1 } ad_relax;
typedef enum { AD_TARGET_PLAIN = 0, AD_TARGET_RESIDUAL = 1 } ad_target;

typedef enum {
    AD_OK = 0,
    AD_EINVAL = 1,      /* bad argument (null pointer, size, alignment, K) */
    AD_EDTYPE = 2,      /* unsupported or mismatched dtype */
    AD_ECALIBER = 3,    /* caliber out of range or K < caliber */
    AD_ESTRUCT = 4,     /* inconsistent sizes (nnz, n) */
    AD_EDEVICE = 5,     /* a HIP runtime call failed */
    AD_ENOMEM = 6,      /* workspace allocation failed */
    AD_EUNSUPPORTED = 7 /* valid request the library does not implement */
} ad_status;

/* sticky device status bits (algdist_status) */
#define AD_STAT_ZERO_DIAG   0x01u /* a row with a zero diagonal was relaxed or used as a residual target */
#define AD_STAT_BAD_COLOR   0x02u /* a colour outside [0, ncolors) was met; such rows were held fixed */
#define AD_STAT_NONFINITE   0x04u /* a distance came out NaN or infinite */
#define AD_STAT_CSR_ROWPTR  0x08u /* csr_validate: row_ptr not nondecreasing or row_ptr[n] != nnz */
#define AD_STAT_CSR_COLS    0x10u /* csr_validate: column out of range or not strictly increasing */
#define AD_STAT_CSR_NODIAG  0x20u /* csr_validate: a row has no diagonal entry */
#define AD_STAT_SEARCH_CAP  0x40u /* ls_interp_search: an F row had more than 64 candidates (row left empty, status 4) */
#define AD_STAT_PATTERN     0x80u /* power_graph_cols: row_ptr_d does not fit A^d's row lengths (rows cut) */
#define AD_STAT_BAD_INTERP  0x100u /* galerkin_*: an interpolation column names a point that is not coarse (ignored) */

typedef struct ad_handle_s *ad_handle;

/* A square sparse matrix in CSR form (device arrays). */
typedef struct {
    int32_t n;              /* rows (= columns), >= 0 */
    int64_t nnz;            /* stored entries, row_ptr[n]; <= INT32_MAX */
    const int32_t *row_ptr; /* [n+1] */
    const int32_t *col;     /* [nnz], sorted per row, diagonal present */
    const void *val;        /* [nnz] float or double, per dtype */
    int32_t dtype;          /* ad_dtype */
} ad_csr;

/* ------------------------------------------------------------------ */
/* handle                                                              */
/* ------------------------------------------------------------------ */

/* Create a handle bound to HIP device `device`.  *h receives the handle. */
int algdist_create(ad_handle *h, int device);

/* Wait for the device, then free the handle and its workspace. */
int algdist_destroy(ad_handle h);

/* Synchronise the handle's device and return the sticky status bits in
 * *bits (host).  clear != 0 resets them to zero afterwards. */
int algdist_status(ad_handle h, uint32_t *bits, int clear);

/* Message describing the last host-side error on this handle ("" if none).
 * The string stays valid until the next call on the handle. */
const char *algdist_last_error(ad_handle h);

int algdist_version(void);

/* Per-kernel timing for measurement.  enable != 0 starts a fresh record:
 * from then on every launch the handle makes is bracketed by two HIP events
 * on its own stream; enable == 0 stops recording.  Kernels are labelled
 * tv_init, color_partition, jacobi, gs_phase, algdist, strength and
 * ls_interp (the last includes its tiny block-sum kernel when ls_sum is
 * requested). */
int algdist_timing(ad_handle h, int enable);

/* Synchronise the device and return the record as text, one line per label:
 * "<label> <launches> <total milliseconds>".  The string stays valid until
 * the next call on the handle. */
const char *algdist_timing_report(ad_handle h);

/* Launch shape of one kernel family, for a (dtype, K, stored-entries-per-row
 * bucket) key.  kernel: "jacobi", "gs_phase", "algdist", "ls_interp",
 * "distance_ls", "batched" (the batch's relaxation stage) or
 * "batched_distance" (the batch's distance stage).  For "algdist" and
 * "batched_distance", lanes_per_row 0 with the plain target and panel rows of
 * at most 128 bytes selects the edge-parallel form (one lane per stored
 * entry).
 * bucket: 0 (< 8 entries per row), 1 (< 16), 2 (< 32), 3 (>= 32), or -1 for
 * all four.  lanes_per_row: lanes sharing one panel row (0 = default; must
 * divide K with K / lanes_per_row entries per lane fitting 64 bytes and
 * being at least 8 bytes).  rows_per_lane: consecutive row steps per
 * workgroup tile (>= 1; ignored by ls_interp, which compacts the F rows of
 * fixed 128-row windows).
 * xcd_map (0 .. 4096): how row tiles map to the 8 XCDs (workgroups are
 * dispatched round-robin over them): 0 = plain block order (consecutive tiles
 * on different XCDs), 1 = one contiguous range of tiles per XCD, c >= 2 =
 * chunks of 8c consecutive tiles with c contiguous tiles per XCD in each.  The kernels' results do not depend on the shape except for the
 * order of the K-reductions inside algdist (all orders stay within the
 * parity bars).  Returns AD_EINVAL for a shape the kernel does not support. */
int algdist_set_launch(ad_handle h, const char *kernel, int32_t dtype, int32_t K, int32_t bucket,
                       int32_t lanes_per_row, int32_t rows_per_lane, int32_t xcd_map);


/* Autotune the launch shapes of this matrix's key (dtype, K, entries-per-row
 * bucket): the relaxation family named by `relax` (color/ncolors as for
 * setup_testvectors), algebraic_distance, and ls_interp (only if cf != NULL
 * and 1 <= caliber <= min(K, 8)).  Every valid (lanes_per_row,
 * rows_per_lane in {1, 2, 4}, xcd_map in {0, 1, 4, 16, 64, 256}) is timed with HIP events on scratch
 * buffers allocated by this call; the fastest is installed as by
 * algdist_set_launch.  cache_json (host path, may be NULL): entries found
 * there for the key are installed without timing; new results are written
 * back (one JSON object per line).  Synchronises the stream. */
int algdist_autotune(ad_handle h, const ad_csr *A, int32_t K, int32_t relax, const int32_t *color,
                     int32_t ncolors, const uint8_t *cf, int32_t caliber, const char *cache_json,
                     void *stream);

/* Time every valid launch shape (lanes per row, row steps per tile, XCD
 * tile mapping) of relax_algdist_batched on this batch (As: host array of
 * nmat device CSRs of one dtype; `sweeps` Jacobi sweeps): first the
 * relaxation stage's shapes, then the distance stage's (including the
 * edge-parallel form), each from its own launches' HIP-event times, and
 * install the fastest of each for the batch's dtype, K and
 * stored-entries-per-row bucket.  cache_json as for algdist_autotune (kernel
 * names "batched" and "batched_distance").  Allocates
 * scratch outputs of the batch's size for the duration of the call and
 * synchronises the stream. */
int algdist_autotune_batched(ad_handle h, int32_t nmat, const ad_csr *As, int32_t K,
                             int32_t sweeps, const char *cache_json, void *stream);

/* Check the CSR invariants listed above on the device; violations set
 * AD_STAT_CSR_* bits.  Not needed on the hot path (no other call reads
 * more than it is given, but their results are defined only for valid
 * CSRs). */
int csr_validate(ad_handle h, const ad_csr *A, void *stream);

/* ------------------------------------------------------------------ */
/* 1. test vectors                                                     */
/* ------------------------------------------------------------------ */

/* Produce K test vectors by relaxation of the homogeneous system A x = 0,
 * each from its own start (Sec. 3, test vectors; Sec. 5.2 relaxes them by
 * Gauss-Seidel).
 *
 * Start: X0 (device, n x K, may be NULL).  When NULL, entry (i, k) is
 * 2u - 1 with u the top 53 bits of output number i*K + k + 1 of splitmix64
 * seeded with `seed`, times 2^-53 (uniform on [-1, 1); rounded to FP32 for
 * an FP32 panel).
 *
 * relax = AD_JACOBI:        x <- x - omega D^{-1} A x, whole vector per sweep.
 * relax = AD_MULTICOLOR_GS: omega is ignored (1).  Per sweep, colours
 *   c = 0..ncolors-1 in turn; a row of colour c becomes x_i - (A z)_i / a_ii
 *   where z_j is the value of this sweep for neighbours of a smaller colour
 *   and the value at the start of the sweep otherwise (same colour included).
 *   This is Gauss-Seidel in colour order for a valid colouring and a
 *   deterministic, race-free rule for any other.  color[n] (device int32);
 *   1 <= ncolors <= 64.
 * Rows with a zero diagonal (AD_STAT_ZERO_DIAG) or a colour outside
 * [0, ncolors) (AD_STAT_BAD_COLOR) are held fixed.
 *
 * Output X (device, n x K) receives x^sweeps.  X must not alias X0.
 * ckpt (device, may be NULL): with ckpt_every = c > 0, receives the iterates
 * x^0, x^c, x^2c, ... (every s < sweeps with s % c == 0) as consecutive
 * n x K panels, ceil(sweeps / c) of them (one, x^0, if sweeps == 0).
 */
int setup_testvectors(ad_handle h, const ad_csr *A, int32_t K, uint64_t seed,
                      const void *X0, int32_t relax, int32_t sweeps, double omega,
                      const int32_t *color, int32_t ncolors,
                      void *X, void *ckpt, int32_t ckpt_every, void *stream);

/* ------------------------------------------------------------------ */
/* 2. algebraic distance (+ fused strength graph)                      */
/* ------------------------------------------------------------------ */

/* For every stored entry (i, j) of A (the diagonal included; Sec. 4.1,
 * eq:measure with j ranging over V_i):
 *     t_i    = x_i                         (target PLAIN, eq:LSfuncrowi), or
 *              x_i - (A x)_i / a_ii        (target RESIDUAL, eq:modls, eq:measure)
 *     p_ij   = <t_i, x_j>_w / <x_j, x_j>_w (0 if x_j = 0)
 *     mu_ij  = sum_k w_k (t_i^k - p_ij x_j^k)^2
 * i.e. mu_ij is the minimum of the one-point least-squares functional and
 * the paper's strength is r_ij = 1 / mu_ij.
 *
 * X: the n x K panel (A's dtype).  w: K FP64 weights (device; NULL = all
 * ones).  mu (device, nnz, A's dtype) receives mu.  p (device, nnz FP64,
 * may be NULL) receives p.  The FP32 path accumulates in FP32 and recomputes
 * in FP64, from the same FP32 inputs, every edge with mu < 1e-4 sum_k w_k t_k^2.
 *
 * Fused strength graph: if strong != NULL (then theta must be in (0, 1)),
 * the strength_graph() outputs below are produced in the same pass.
 */
int algebraic_distance(ad_handle h, const ad_csr *A, int32_t K, const void *X,
                       const double *w, int32_t target, void *mu, double *p,
                       double theta, const uint8_t *fmask, uint8_t *strong,
                       int32_t *nstrong, void *stream);

/* ------------------------------------------------------------------ */
/* 3. strength graph                                                   */
/* ------------------------------------------------------------------ */

/* Sec. 4.2, eq:strength_graph: for i in F the edge (i, j), j in F, j != i,
 * is strong iff r_ij > theta max_k r_ik (k over the row's F-neighbours,
 * k != i), r = 1/mu.  Evaluated division-free in FP64 as
 *     m_i > theta mu_ij  with m_i = min_k mu_ik,
 * and, when m_i = 0, exactly the edges with mu_ij = 0 are strong.
 * fmask (device, n bytes, may be NULL = all rows in F): nonzero marks F.
 * strong (device, nnz bytes) receives 0/1 (0 on the diagonal and outside
 * F); nstrong (device, n int32, may be NULL) the per-row count.
 * 0 < theta < 1. */
int strength_graph(ad_handle h, const ad_csr *A, const void *mu, double theta,
                   const uint8_t *fmask, uint8_t *strong, int32_t *nstrong, void *stream);

/* ------------------------------------------------------------------ */
/* 4. least-squares interpolation                                      */
/* ------------------------------------------------------------------ */

/* Sec. 3.1, eq:LSfuncrowi (target PLAIN) / eq:modls (target RESIDUAL): for
 * each F row i (cf[i] == 0) the row p_i minimising
 *     sum_k w_k (t_i^k - sum_{j in C_i} p_ij x_j^k)^2,
 * with C_i the (at most) `caliber` C-neighbours (cf[j] != 0, j != i,
 * a_ij stored) of smallest mu_ij, ties to the lower column -- the
 * one-sided-distance scan the final remark of Sec. 4.3 describes.
 * The normal equations are formed and solved in FP64 (Cholesky), also for
 * an FP32 panel.  Columns are taken in increasing-mu order; one whose pivot
 * is <= 1e-12 times its Gram diagonal (numerically in the span of those
 * kept) is dropped.
 *
 * Outputs (device, row-major n x caliber for P):
 *   P_col:  fine column index of each weight, in increasing-mu order,
 *           -1 padded; C rows: P_col[i][0] = i.
 *   P_val:  FP64 weights (0 padded); C rows: 1.
 *   ls_val: FP64 functional at the minimiser (0 for C rows).
 *   row_status: 0 ok, 1 F row without C-neighbour (empty row, ls_val =
 *           sum w t^2), 2 a column was dropped, 3 residual target with a
 *           zero diagonal (plain target used).
 *   ls_sum (may be NULL): one FP64, the sum of ls_val over F rows, summed
 *           in a fixed order (run-to-run identical).
 * 1 <= caliber <= 8 and caliber <= K (the uniqueness remark of Sec. 3.1).
 * mu is A's dtype (as produced by algebraic_distance).
 */
int ls_interp(ad_handle h, const ad_csr *A, int32_t K, const void *X, const double *w,
              const uint8_t *cf, const void *mu, int32_t caliber, int32_t target,
              int32_t *P_col, double *P_val, double *ls_val, int32_t *row_status,
              double *ls_sum, void *stream);

/* The distances with the fused strength row (algebraic_distance with
 * p = NULL) and the LS rows on them (ls_interp) in one pass over the rows:
 * each row's entries, distances and panel rows are read once for both.
 * Arguments as in those two calls (mu is written here and read by nothing
 * else); strong / nstrong may be NULL (no strength row), fmask may be NULL.
 * The row-group form with lanes_per_row L (algdist_set_launch("distance_ls",
 * ...), default 16 bytes of panel per lane, or algdist_autotune) gives, for
 * every row, bitwise the mu, mask and LS row of algebraic_distance and
 * ls_interp run with the same L; ls_sum may differ from ls_interp's in the
 * last bits (another order of the FP64 block partial sums).
 * Uses handle workspace for the block partial sums when ls_sum is given. */
int distance_ls(ad_handle h, const ad_csr *A, int32_t K, const void *X, const double *w,
                int32_t target, void *mu, double theta, const uint8_t *fmask, uint8_t *strong,
                int32_t *nstrong, const uint8_t *cf, int32_t caliber, int32_t *P_col,
                double *P_val, double *ls_val, int32_t *row_status, double *ls_sum, void *stream);

/* distance_ls for callers that cannot allocate device memory (code under
 * graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, same kernels and bitwise the same results as distance_ls,
 * but it never allocates or frees.  The per-workgroup partial sums of ls_sum
 * go to a static device array of 1 MiB (131072 FP64 values; each device the
 * library runs on holds one until the process ends), resolved once per
 * device by algdist_create.  A call whose fused pass would launch more
 * than 131072 workgroups with ls_sum requested (FP32, K = 16 at the default
 * launch shape of 64 rows per workgroup: more than about 8.3 million rows)
 * returns AD_ESTRUCT and enqueues nothing; without ls_sum there is no
 * limit.  Every call on one
 * device shares that array, so calls that overlap in time on one device
 * (any handle, any stream) race; the array needs no clearing (each call
 * writes every partial it reads). */
int distance_ls_noalloc(ad_handle h, const ad_csr *A, int32_t K, const void *X, const double *w,
                        int32_t target, void *mu, double theta, const uint8_t *fmask,
                        uint8_t *strong, int32_t *nstrong, const uint8_t *cf, int32_t caliber,
                        int32_t *P_col, double *P_val, double *ls_val, int32_t *row_status,
                        double *ls_sum, void *stream);

/* ------------------------------------------------------------------ */
/* long-range connectivity and the search over interpolatory sets      */
/* ------------------------------------------------------------------ */

/* Pattern of A^d, d >= 1 (Sec. 4.1, eq. graph: V_i = {j : (A^d)_ij != 0};
 * the closing remark of Sec. 4.2: A^d is never formed, its graph is rebuilt
 * from the graph of A).  Read structurally: row i holds every j joined to i
 * by a walk of exactly d steps -- with every diagonal stored, every j within
 * graph distance d -- in increasing order; cancellation in A^d's values is
 * ignored.  Only A's structure is read (A->val may be NULL).
 *
 * power_graph_rows writes the row pointers row_ptr_d (device, n + 1 int32)
 * and the entry count *nnz_d (host); it synchronises `stream`, so it cannot
 * be captured.  Returns AD_EUNSUPPORTED when a row would have more than
 * 1024 entries or the count would pass INT32_MAX (row_ptr_d is then
 * undefined).  power_graph_cols then writes the sorted columns col_d
 * (device, *nnz_d int32) for those row pointers, asynchronously.  The pair
 * (row_ptr_d, col_d) is the pattern argument of algebraic_distance_graph
 * and ls_interp_search. */
int power_graph_rows(ad_handle h, const ad_csr *A, int32_t d, int32_t *row_ptr_d,
                     int64_t *nnz_d, void *stream);
int power_graph_cols(ad_handle h, const ad_csr *A, int32_t d, const int32_t *row_ptr_d,
                     int32_t *col_d, void *stream);

/* algebraic_distance over the entries of another pattern G of the same n
 * rows -- typically that of A^d from power_graph_* (Sec. 4.1: mu_ij for all
 * j in V_i of G_d; Sec. 4.2 builds the strength graph M^d on it).  The target
 * t_i is formed from A (plain x_i, or x_i - (A x)_i / a_ii), the one-point
 * fit runs against every x_j, j in row i of G.  G: row_ptr_g (n + 1 int32),
 * col_g (nnz_g int32, sorted per row; the diagonal is not required).  mu, p,
 * strong (nnz_g) are per entry of G; nstrong per row; theta, fmask, w as
 * in algebraic_distance (the strength graph is that of Sec. 4.2 on G). */
int algebraic_distance_graph(ad_handle h, const ad_csr *A, int64_t nnz_g,
                             const int32_t *row_ptr_g, const int32_t *col_g, int32_t K,
                             const void *X, const double *w, int32_t target, void *mu, double *p,
                             double theta, const uint8_t *fmask, uint8_t *strong,
                             int32_t *nstrong, void *stream);

/* Interpolatory sets by search (Sec. 4.3).  For each F row i (cf[i] == 0)
 * the candidates are N_i = the C-points (cf != 0) of row i of the pattern G
 * (eq:nbhd with G the pattern of A^{d_LS}), i excluded.  Every set W within
 * N_i with 1 <= |W| <= caliber is fitted (the LS functional of Sec. 3.1,
 * eq:LSfuncrowi or eq:modls per target, weights w): its minimiser by a
 * Cholesky of its Gram matrix, its functional by definition from the
 * residual; a set whose Gram matrix has a Cholesky pivot <= 1e-8 of its
 * diagonal (a column with a part independent of the earlier ones below
 * 1e-4 of its norm) is numerically dependent and skipped.  For each size m
 * the set of least functional best_m is kept (ties: the first in
 * lexicographic order of candidate positions).  The size follows the penalty rule of Sec. 4.3 read as a scan
 * in increasing size against the incumbent, on values relative to the
 * empty set's S = sum_k w_k t_k^2: the incumbent starts at the smallest size
 * with a fitted set and is replaced by size m when
 *     best_m / S < (incumbent / S)^(gamma (m - incumbent size)).
 * The paper's gamma is 1.5.  Outputs as in ls_interp: P_col (the chosen W in
 * increasing column order, -1 padded; C rows: i), P_val (FP64 minimiser),
 * ls_val (functional at it, by definition), row_status: 0 ok, 1 no
 * candidate (or all dependent; ls_val = S), 3 residual target with a zero
 * diagonal (plain target used), 4 more than 64 candidates (row left empty;
 * AD_STAT_SEARCH_CAP set).  1 <= caliber <= min(4, K).  Work per F row grows
 * as |N_i|^caliber; G's rows may hold up to 1024 entries. */
int ls_interp_search(ad_handle h, const ad_csr *A, int64_t nnz_g, const int32_t *row_ptr_g,
                     const int32_t *col_g, int32_t K, const void *X, const double *w,
                     const uint8_t *cf, int32_t caliber, double gamma, int32_t target,
                     int32_t *P_col, double *P_val, double *ls_val, int32_t *row_status,
                     void *stream);

/* ------------------------------------------------------------------ */
/* batched relaxation + distances                                      */
/* ------------------------------------------------------------------ */

/* For each of nmat matrices As[m] (host array of device CSRs, one dtype):
 * the test-vector start, `sweeps` damped-Jacobi sweeps with omega
 * (relax = AD_JACOBI; AD_MULTICOLOR_GS returns AD_EUNSUPPORTED: a batch
 * carries no colouring), and the
 * distances of Sec. 4.1 (plain target) with the fused strength graph of
 * Sec. 4.2 (theta; all rows in F) -- exactly what setup_testvectors +
 * algebraic_distance compute for the block-diagonal matrix made of the
 * batch.
 * Outputs are concatenated in matrix order: X (sum n) x K, mu (sum nnz,
 * the CSR's dtype), strong (sum nnz, may be NULL), nstrong (sum n, may be
 * NULL).  Start values use the global row index: entry (r, k) of the
 * concatenated panel is the (r*K + k + 1)-th splitmix64 output from seed.
 * w (K FP64, may be NULL) weights the distances.
 * Every member is cut into row tiles; each stage (start, each sweep,
 * distances) is one launch over the tiles of all members, so no workgroup
 * waits on another.  The first call for a given argument set (pointers,
 * sizes, scalars, launch shape) uploads the tile table and captures the
 * sweeps + 2 launches in a HIP graph; later calls with the same arguments
 * replay it on `stream`.  With per-kernel timing on, or when the caller is
 * capturing `stream`, the launches are issued directly instead.  The batch
 * state (a second panel of (sum n) x K, the tables, the graph) is owned by
 * the handle and freed by algdist_destroy.  Calls that overlap on one
 * handle race.  Launch shapes: algdist_set_launch("batched", ...) for the
 * relaxation stage and ("batched_distance", ...) for the distance stage, or
 * algdist_autotune_batched. */
int relax_algdist_batched(ad_handle h, int32_t nmat, const ad_csr *As, int32_t K, uint64_t seed,
                          int32_t relax, int32_t sweeps, double omega, const double *w, void *X,
                          void *mu, double theta, uint8_t *strong, int32_t *nstrong, void *stream);

/* ------------------------------------------------------------------ */
/* adjoint of the LS interpolation loss                                */
/* ------------------------------------------------------------------ */

/* Gradient of L = sum_{i in F} ls_val_i, where ls_val is the plain-target LS
 * functional of Sec. 3.1 (eq:LSfuncrowi) at the rows p fitted to
 * x^S = J^S x^0, J x = x - omega D^{-1} A x (damped Jacobi, Sec. 3 test
 * vectors), with respect to the stored values of A and to omega.
 * Because each p_i minimises its row's functional, L's dependence through p
 * vanishes to first order and p enters as fixed weights.  The chain rule
 * runs the sweeps backward: y = D^{-1} g, dL/da_ij -= omega <y_i, x_j^s>,
 * dL/da_ii += omega <y_i, (A x^s)_i> / a_ii, dL/domega -= <y, A x^s>,
 * g <- g - omega A^T y, from the seed g = dL/dx^S.
 *
 * FP64 only (A->dtype == AD_F64).  Any sparsity pattern: the products with
 * A^T and P^T gather through a column-major index of the pattern that the
 * call builds in the handle's workspace.  1 <= caliber <= min(8, K).
 * Inputs (device): ckpt, the iterates x^0, x^c, x^2c, ... written by
 * setup_testvectors with ckpt_every = c (others are recomputed forward);
 * X_final = x^S; w (K, may be NULL); cf; P_col / P_val (n x caliber) from
 * ls_interp on X_final with the plain target; dL, one FP64 (the upstream
 * derivative, e.g. 1.0).
 * Outputs (device): grad_val (nnz FP64, overwritten), grad_omega (one FP64).
 * Uses handle workspace of about (4 + c) n K doubles + nnz ints.
 */
int ls_interp_loss_backward(ad_handle h, const ad_csr *A, int32_t K, const void *ckpt,
                            int32_t ckpt_every, int32_t sweeps, double omega, const double *w,
                            const uint8_t *cf, const int32_t *P_col, const double *P_val,
                            int32_t caliber, const void *X_final, const double *dL,
                            double *grad_val, double *grad_omega, void *stream);

/* The gradient of the same loss for test vectors relaxed by either rule of
 * setup_testvectors, and with respect to the LS weights as well.
 * relax = AD_JACOBI: as ls_interp_loss_backward (grad_omega may be NULL).
 * relax = AD_MULTICOLOR_GS (color/ncolors as for setup_testvectors, omega
 * ignored; grad_omega, if given, receives 0): one colour phase is the map
 * v' = v - E_c D^{-1} A v (E_c: the rows of colour c), its adjoint is
 * g = g' - A^T y with y = D^{-1} E_c g', and it adds -<y_i, v_j> to
 * dL/da_ij and <y_i, (A v)_i> / a_ii to dL/da_ii; a sweep's phases are
 * undone in reverse colour order, their states recomputed from the sweep's
 * iterate.  grad_w (device, K FP64, may be NULL) receives dL/dw_k = dL *
 * sum over F rows of (x_i^k - sum_j p_ij x_j^k)^2 at X_final (p minimises
 * each row's functional, so its own variation does not enter; Sec. 3.1
 * eq:LSfuncrowi).  Other arguments as for ls_interp_loss_backward; ckpt
 * comes from setup_testvectors with the same relax and colouring.  Uses
 * handle workspace of about (4 + c + ncolors) n K doubles + nnz ints. */
int ls_interp_loss_grad(ad_handle h, const ad_csr *A, int32_t K, int32_t relax,
                        const int32_t *color, int32_t ncolors, const void *ckpt,
                        int32_t ckpt_every, int32_t sweeps, double omega, const double *w,
                        const uint8_t *cf, const int32_t *P_col, const double *P_val,
                        int32_t caliber, const void *X_final, const double *dL, double *grad_val,
                        double *grad_omega, double *grad_w, void *stream);

/* ------------------------------------------------------------------ */
/* Compatible-relaxation coarsening (Sec. 3.2; Sec. 4.2, Algorithm 1).  */
/* These calls are synchronous (the host decides between stages and     */
/* rounds), allocate their own device buffers, and must not be made     */
/* while `stream` is capturing.                                         */
/* ------------------------------------------------------------------ */

/* One CR run (eq:frelax, eq:meas1): nu >= 1 sweeps of F-relaxation of the
 * homogeneous system from the constant start (1 on F, 0 on C; cf[i] != 0
 * marks C), the relaxation being the colour-phase Gauss-Seidel of
 * setup_testvectors restricted to F (C rows take no colour and stay at 0).
 * color/ncolors as for setup_testvectors (rows with an invalid colour are
 * held as well).
 * Outputs: u (device, n values of A's dtype, may be NULL) = u^nu; *rho (host)
 * = (||u_f^nu||_2 / ||u_f^0||_2)^(1/nu), 0 when F is empty; norms (host, 3
 * doubles, may be NULL) = |F|, sum over F of (u_i^nu)^2, max over F of
 * |u_i^nu|, all accumulated in FP64. */
int cr_rate(ad_handle h, const ad_csr *A, const int32_t *color, int32_t ncolors,
            const uint8_t *cf, int32_t nu, void *u, double *rho, double *norms, void *stream);

/* Candidate set of Algorithm 1 with the measure of the remark after it:
 * z[i] = 1 (device, n bytes) for the F points (cf[i] == 0) with
 * |u_i| / max over F of |u| > tol, compared in FP64; u (device, n values of
 * type dtype). */
int cr_candidates(ad_handle h, int32_t n, int32_t dtype, const uint8_t *cf, const void *u,
                  double tol, uint8_t *z, void *stream);

/* Independent set of the candidates z (device, n bytes) on the strength
 * graph (Algorithm 1): strong (device, nnz bytes) marks entry (i, j) of A's
 * pattern; candidates i and j are neighbours when strong(i, j) or
 * strong(j, i).  The set is the greedy maximal one in decreasing
 * (lambda_i, h_i, i), lambda_i = |S_i^T| (strong entries in column i, the
 * weight of the classical colouring of Sec. 2), h_i the (i+1)-th output of
 * splitmix64 seeded with `seed`; it is found by parallel rounds of local
 * maxima, which give exactly that set.  sel (device, n bytes) receives 0/1;
 * *count (host, may be NULL) its size.  Only A's pattern is used. */
int independent_set(ad_handle h, const ad_csr *A, const uint8_t *strong, const uint8_t *z,
                    uint64_t seed, uint8_t *sel, int64_t *count, void *stream);

/* Algorithm 1: from C_0 (cf, device n bytes, in/out; cf[i] != 0 marks C),
 * run cr_rate; while rho_f > delta: candidates with tol = 1 - rho_f, the
 * strength graph (strength_graph on mu with the F mask, i.e. restricted to
 * F), C grown by the independent set of the candidates with seed
 * seed + stage, and cr_rate again.  Stops also when a stage adds nothing or
 * after max_stages stages.  Outputs (host): rho[s], ncoarse[s] = rho_f and
 * |C| after s stages (arrays of max_stages + 1), *nstages = stages run.
 * mu: nnz distances of A's dtype (algebraic_distance on the test vectors).
 * The paper's parameters are nu = 5, delta = 0.7 (Sec. 5.2). */
int cr_coarsening(ad_handle h, const ad_csr *A, const int32_t *color, int32_t ncolors,
                  const void *mu, double theta, int32_t nu, double delta, int32_t max_stages,
                  uint64_t seed, uint8_t *cf, double *rho, int64_t *ncoarse, int32_t *nstages,
                  void *stream);

/* cr_coarsening with the strength graph M^d of Sec. 4.2: the strength
 * graph and the independent set live on the pattern G (row_ptr_g [n+1],
 * col_g [nnz_g], device, rows sorted; e.g. from power_graph_rows /
 * power_graph_cols for the graph of A^d) with mu_g one distance per entry
 * of G in A's dtype (e.g. from algebraic_distance_graph); the F-relaxation
 * sweeps and rho_f use A.  Arguments, outputs, synchronisation and errors
 * as cr_coarsening; G = A's pattern gives cr_coarsening's result. */
int cr_coarsening_graph(ad_handle h, const ad_csr *A, int64_t nnz_g, const int32_t *row_ptr_g,
                        const int32_t *col_g, const int32_t *color, int32_t ncolors,
                        const void *mu_g, double theta, int32_t nu, double delta,
                        int32_t max_stages, uint64_t seed, uint8_t *cf, double *rho,
                        int64_t *ncoarse, int32_t *nstages, void *stream);

/* ------------------------------------------------------------------ */
/* Galerkin coarse operator and the two-grid method (Sec. 5.2).          */
/* Synchronous; the calls allocate their own device buffers.            */
/* ------------------------------------------------------------------ */

/* Interpolation P (n x nc) in the layout ls_interp / ls_interp_search
 * write: P_col (device, n x caliber int32, fine indices of C points, -1
 * padded; a C row names itself), P_val (device, n x caliber FP64).  The C
 * points (cf[i] != 0) are numbered in increasing fine index.  A column
 * naming a non-C point or an index outside [0, n) is ignored and sets
 * AD_STAT_BAD_INTERP.
 *
 * A_c = P^T A P.  Coarse row I accumulates (p_iI * a_ij) * p_jJ over the
 * fine rows i of column I of P in increasing i (then stored slot), row i's
 * entries in CSR order and row j's slots in order, each product and sum
 * rounded separately: the coefficients are those of that plain loop,
 * bit for bit.  Every column reached by a product is stored (also when the
 * products cancel), sorted ascending.
 *
 * galerkin_rows: *nc (host) = number of C points; row_ptr_c (device, room
 * for n + 1 int32) receives nc + 1 row pointers; *nnz_c (host) the number
 * of entries.  AD_EUNSUPPORTED when a coarse row has more than 64
 * contributing fine rows or more than 2048 products, or nnz_c > 2^31 - 1.
 * galerkin_cols then writes col_c (nnz_c int32) and val_c (nnz_c FP64). */
int galerkin_rows(ad_handle h, const ad_csr *A, int32_t caliber, const int32_t *P_col,
                  const double *P_val, const uint8_t *cf, int32_t *nc, int32_t *row_ptr_c,
                  int64_t *nnz_c, void *stream);
int galerkin_cols(ad_handle h, const ad_csr *A, int32_t caliber, const int32_t *P_col,
                  const double *P_val, const uint8_t *cf, int32_t nc, const int32_t *row_ptr_c,
                  int32_t *col_c, double *val_c, void *stream);

/* The two-grid method of Sec. 5.2 on the homogeneous system A e = 0, for
 * the K columns of E0 (device, n x K FP64, e.g. random starts) at once:
 * per cycle `pre` colour-phase Gauss-Seidel sweeps (setup_testvectors'
 * rule; color/ncolors as there), e <- e - P A_c^{-1} P^T A e with A_c
 * (nc rows, from galerkin_*) factored once by dense Cholesky (the direct
 * coarse solve; nc <= 8192), `post` sweeps.  hist (host, may be NULL,
 * (iters + 1) x K) receives ||e^t||_A; rho (host, K) = ||e^iters||_A /
 * ||e^(iters-1)||_A.  FP64 only.  AD_ESTRUCT if A_c is not positive
 * definite.  The paper's settings: iters = 100, pre = post = 2. */
int two_grid_rate(ad_handle h, const ad_csr *A, const int32_t *color, int32_t ncolors,
                  int32_t caliber, const int32_t *P_col, const double *P_val, const uint8_t *cf,
                  int32_t nc, const int32_t *row_ptr_c, const int32_t *col_c, const double *val_c,
                  int32_t K, const void *E0, int32_t iters, int32_t pre, int32_t post,
                  double *hist, double *rho, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* ALGDIST_H */
