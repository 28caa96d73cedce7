/*
 * flp.h - filtered Lanczos procedure on MI355X (gfx950): C ABI.
 *
 * Computes every eigenpair of a large sparse real symmetric matrix A that
 * lies in a closed interval [alpha, beta] (the problem stated in the
 * paper's program summary), by Lanczos on a Chebyshev polynomial filter
 * p(A) of the interval's indicator (Sections 2.2-2.3), following
 * Aurentz, Kalantzis and Saad, "Cucheb: a GPU implementation of the
 * filtered Lanczos procedure".
 *
 * Conventions shared by every call
 * --------------------------------
 * - Return value: 0 (FLP_OK) on success, a negative FLP_E_* code otherwise.
 *   On failure flp_last_error() returns a message (thread-local).  No C++
 *   exception crosses this boundary.
 * - Device pointers are hipMalloc'd (or torch-allocated) memory on the
 *   current HIP device; host pointers are ordinary memory.  Each argument
 *   below says which.
 * - Blocks of r vectors are row-major n x r: entry (i, j) at [i * ld + j],
 *   ld >= r.  The matrix is CSR, zero-based int32 indices, columns sorted
 *   within a row, both triangles stored (Section 3.2.1 keeps the full
 *   symmetric matrix on the GPU without exploiting symmetry).
 * - `stream` is a hipStream_t passed as void*; NULL means the default
 *   stream.
 * - The library keeps a workspace per calling thread and device that grows
 *   on demand and is released by flp_release_workspace() (the calling
 *   thread's) or when the thread ends.  Calls from one thread share its
 *   workspace, so asynchronous calls from one thread on different streams
 *   must not overlap in time; calls from different threads do not share
 *   it.
 */
#ifndef FLP_H
#define FLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ errors */
#define FLP_OK            0
#define FLP_E_ARG        -1  /* invalid argument (NaN, alpha >= beta, r < 1, n <= 0, ...) */
#define FLP_E_INTERVAL   -2  /* [alpha, beta] does not meet [lambda_min, lambda_max] */
#define FLP_E_NOTSYM     -3  /* matrix failed the optional symmetry check */
#define FLP_E_NOMEM      -4  /* device allocation failed or exceeds the limit */
#define FLP_E_NOCONV     -5  /* basis limit reached before convergence (result still returned) */
#define FLP_E_DEVICE     -6  /* HIP runtime error; message in flp_last_error() */
#define FLP_E_PENDING    -7  /* serving: the request has not finished yet (flp_server_poll) */
#define FLP_E_CANCELLED  -8  /* serving: the request was cancelled (flp_server_cancel) */

/* precision of the filter recurrence (Section 2.2 applies p(A) by Clenshaw) */
#define FLP_PREC_FP64         0  /* FP64 matrix values, vectors and accumulation */
#define FLP_PREC_FP32_FILTER  1  /* FP32 values/vectors/accumulation in the filter only */

/* storage formats of the filter's SpMMs (flp_opts.format) */
#define FLP_FORMAT_AUTO 0
#define FLP_FORMAT_CSR 1
#define FLP_FORMAT_SELL 2

/* ------------------------------------------------------------------ types */

/* Sparse symmetric matrix in CSR form (Section 3.2.1).  All pointers are
 * DEVICE pointers owned by the caller, who keeps them alive until every
 * call using them has completed.  val32 is optional: an FP32 copy of val
 * used by FLP_PREC_FP32_FILTER (the library converts val itself when it is
 * NULL). */
typedef struct flp_csr {
    int32_t n;              /* order of A, > 0 */
    int64_t nnz;            /* stored entries, < 2^31 */
    const int32_t *rowptr;  /* device int32[n + 1], rowptr[0] = 0, non-decreasing */
    const int32_t *colind;  /* device int32[nnz], 0 <= colind < n */
    const double *val;      /* device float64[nnz] */
    const float *val32;     /* device float32[nnz] or NULL */
} flp_csr;

/* A Chebyshev filter polynomial (Section 3.2.3 stores the degree, the
 * Chebyshev coefficients and the spectrum bounds).  Opaque; host memory. */
typedef struct flp_filter flp_filter;

/* Options for flp_solve.  Fill with flp_opts_default() first. */
typedef struct flp_opts {
    int32_t block;        /* block size r >= 1 (Section 2.3); default 1 */
    int32_t degree;       /* filter degree m; <= 0 selects it by eq. optimaldegree */
    double eps;           /* tolerance of the degree rule; default 0.31227 */
    double tol;           /* required ||Ax - lambda x|| / ||A||; default 1e-9 */
    int32_t check_every;  /* block steps between convergence checks; <= 0 (default) picks
                             min(30, round(90 / block)): the paper's spacing of 90 basis
                             columns (30 steps at block size 3), at most 30 steps */
    int32_t prec;         /* FLP_PREC_FP64 (default) or FLP_PREC_FP32_FILTER */
    uint64_t seed;        /* seed of the random start block and bounds start vector */
    int64_t max_basis;    /* cap on Lanczos basis columns; <= 0 picks min(n, memory) */
    int32_t k0;           /* Lanczos steps of the bounds estimate; default 40 */
    const double *start;  /* HOST n x block row-major start block, or NULL (random) */
    double lmin, lmax;    /* spectrum bounds to use if lmin < lmax; else estimated */
    void *stream;         /* hipStream_t, NULL = default stream */
    double sym_tol;       /* >= 0: run flp_check_symmetric(A, sym_tol) first; < 0 (default): skip */
    int32_t polish_degree;  /* FP32 filter only: degree of the FP64 polish filter on the same
                               interval; <= 0 (default) uses the solve's degree */
    int32_t unfiltered;   /* 1: plain block Lanczos with Ahat itself in place of p(Ahat) (the
                             unfiltered Lanczos that Section 4.1 sets beside the filtered one); FP64 only and flp_solve
                             only (FLP_E_ARG elsewhere).  Ritz values of Ahat inside the
                             mapped interval, and the nearest one outside on each side, must
                             converge; max_basis <= 0 then means min(n, 12288). */
    int32_t format;       /* storage the filter's SpMMs read A in: FLP_FORMAT_CSR, FLP_FORMAT_SELL
                             (a sliced ELL copy built at set-up: slices of 64 rows padded to
                             their longest row, column-major inside a slice; the "other
                             sparse formats" of Section 5), or FLP_FORMAT_AUTO (default):
                             SELL unless padding would add more than 25 % to the stored
                             entries.  Results are bit-identical either way.  Each solve
                             builds its own copy (device memory about that of A's column
                             indices and values), also in the batched and serving forms;
                             flp_solve_sliced keeps CSR (its slices share A) and refuses SELL
                             with FLP_E_ARG. */
    const double *warm;   /* flp_solve only: DEVICE n x warm_count column-major (the layout of
                             flp_result.evecs), or NULL.  Warm start for a sequence of related
                             problems (the self-consistent-field loops of Section 1: each matrix
                             a small change of the previous one): the previous eigenvectors
                             and warm_count / 2 (at least 2 block) random guard columns are
                             refined by subspace iteration with the filter (each sweep
                             X <- p(Ahat) X in FP64 accuracy by the residual form, orthonormalise,
                             Rayleigh-Ritz with A; degree max(polish_degree or degree, 20))
                             instead of a Lanczos run.  It stops when every Ritz pair inside
                             [alpha, beta] meets tol, their count did not change since the
                             previous sweep, and at least two Ritz pairs outside the interval
                             have settled (residual <= 1e-4 ||A||) on values whose filter value
                             is below the candidate threshold tau (the block reaches past the
                             interval's transition band, so no eigenvalue inside is left out).
                             While no guard gets past the band the guards are doubled, at most
                             twice; after 16 sweeps the call falls back to the cold solve.
                             stats.warm_status says which ran. */
    int32_t warm_count;   /* columns of warm (0: cold start) */
} flp_opts;

typedef struct flp_stats {
    int32_t iters;         /* block Lanczos steps behind the result (the paper's "iters") */
    int64_t mv;            /* products with A inside the filter: r * m * (block steps taken),
                              which may exceed r * m * iters by the few steps taken while
                              the deciding convergence check ran on the host */
    int32_t basis_cols;    /* Lanczos basis columns at convergence */
    int32_t polish_sweeps; /* FP64 refinement sweeps (FP32 filter only) */
    double t_pre;          /* seconds: spectrum bounds (the paper's PREPROC) */
    double t_mv;           /* seconds: filter applications (the paper's MV) */
    double t_orth;         /* seconds: reorthogonalisation + block QR (ORTH) */
    double t_check;        /* seconds: convergence checks (host eigensolves) */
    double t_rr;           /* seconds: Rayleigh-Ritz, residuals, polish */
    double t_total;        /* seconds: whole call */
    double filter_bytes;   /* algorithmic bytes moved by the filter SpMMs */
    double orth_bytes;     /* algorithmic bytes of the reorthogonalisation: the basis
                              (n x k doubles) read twice per Gram-Schmidt pass */
    int32_t filter_format; /* storage the filter read A in: FLP_FORMAT_CSR or FLP_FORMAT_SELL */
    int32_t filter_group_width;     /* filter launch configuration of a single solve (0 in
                                       batched and serving results): columns per launch, */
    int32_t filter_lanes_per_row;   /* lanes per matrix row, */
    int32_t filter_cols_per_lane;   /* columns per lane and */
    int32_t filter_streaming_loads; /* nontemporal loads of V and U_{k+2} (1) or not (0) and */
    int32_t filter_tile_chunk;      /* the tile-to-XCD mapping (flp_tune_info.tile_chunk) */
    double polish_bytes;   /* FP32 filter only: algorithmic bytes of the residual-form polish
                              sweeps (not part of filter_bytes) */
    double t_polish;       /* seconds: those sweeps' device time (part of t_rr, not of t_mv) */
    int32_t warm_status;   /* 0: cold solve; 1: the warm start's result; 2: the warm start could
                              not certify its result and the cold solve ran */
    int32_t warm_sweeps;   /* subspace iteration sweeps of the warm start (polish_sweeps counts
                              them too when it was used) */
    int32_t filter_lds_window; /* single solve's filter: its LDS window (flp_tune_info.lds_window:
                                  0 none, 1 fixed +-8 rows, 2 sliding) */
    int32_t filter_window_halo; /* its reach in rows (flp_tune_info.window_halo) */
    int32_t separations;        /* FP32 filter: Rayleigh-Ritz rounds on a block grown by A x for Ritz
                                   pairs mixing eigenvectors from both sides of the interval */
    int32_t candidates;         /* Ritz pairs of the last check with filter value >= tau (the
                                   candidates of eq. proj) */
    int32_t guards;             /* FP32 filter: transition-band Ritz vectors added to them for the
                                   polish (0 otherwise) */
} flp_stats;

/* Result of flp_solve; owned by the library until flp_result_free(). */
typedef struct flp_result {
    int32_t n;
    int32_t count;        /* eigenvalues found in [alpha, beta], with multiplicity */
    double *evals;        /* HOST float64[count], ascending */
    double *resid;        /* HOST float64[count]: ||A x - lambda x||_2 / ||A|| */
    double *evecs;        /* DEVICE float64[n * count], column-major (x_j at evecs + j*n) */
    double lmin, lmax;    /* spectrum bounds used for the affine map (eq. transf) */
    double alpha, beta;   /* the interval as given */
    int32_t degree;       /* filter degree used */
    int32_t converged;    /* 1 if the stopping rule was met and every returned pair has
                             resid <= opts.tol (else the call returns FLP_E_NOCONV) */
    flp_stats stats;
} flp_result;

/* ------------------------------------------------------------------ calls */

/* Fill *o with the defaults listed in flp_opts. */
void flp_opts_default(flp_opts *o);

/* Build the filter p_m = sum_{i<=m} b_i T_i for the indicator of
 * [alpha, beta] (Section 2.2: closed-form Chebyshev coefficients of the
 * ideal filter phi; truncation at degree m).
 *   alpha, beta: the interval in A's units, alpha < beta.
 *   degree: m >= 1, or <= 0 to pick the smallest m with
 *           ||p_m - phi|| < eps ||phi|| (eq. optimaldegree, eps = 0.31227).
 *   lmin, lmax: bounds of A's spectrum, lmin < lmax; the map
 *           A -> (A - cI)/e of eq. transf uses c = (lmin+lmax)/2,
 *           e = (lmax-lmin)/2.  Pass -1, 1 when alpha, beta are already
 *           in [-1, 1].  [alpha, beta] is clamped to [lmin, lmax].
 *   out: receives a new filter (host memory); free with flp_filter_free.
 * Errors: FLP_E_ARG (NaN, alpha >= beta, lmin >= lmax, degree > 100000),
 *         FLP_E_INTERVAL (empty after clamping). */
int flp_build_filter(double alpha, double beta, int32_t degree, double lmin, double lmax,
                     flp_filter **out);
int flp_build_filter_eps(double alpha, double beta, int32_t degree, double lmin, double lmax,
                         double eps, flp_filter **out);
void flp_filter_free(flp_filter *p);
/* Degree m of the filter. */
int32_t flp_filter_degree(const flp_filter *p);
/* Copy b_0..b_m into host coeffs[0..cap); returns m + 1 (or a negative error). */
int32_t flp_filter_coeffs(const flp_filter *p, double *coeffs, int32_t cap);
/* Spectrum bounds and mapped interval: out[0..5] = lmin, lmax, c, e, alpha', beta'. */
int flp_filter_info(const flp_filter *p, double *out6);
/* Evaluate p at host points z (already in [-1,1] units), host in/out. */
int flp_filter_eval(const flp_filter *p, const double *z, double *out, int32_t count);
/* Chebyshev coefficients c_0..c_{m-1} of g(z) = (p(z) - p(t)) / (z - t), the
 * divided difference of the filter at t (in [-1,1] units), into host
 * coeffs[0..cap); returns m (or a negative error).  The FP32-filter polish
 * applies g to each Ritz vector's residual: p(Ahat) x = p(t) x + g(Ahat) r
 * when Ahat x = t x + r. */
int32_t flp_filter_divided(const flp_filter *p, double t, double *coeffs, int32_t cap);

/* W = p(Ahat) V, Ahat = (A - cI)/e (eq. transf), by Clenshaw's backward
 * recurrence (Section 2.2) with the affine map and the three-term update
 * fused into each sparse-matrix product: m products with A.
 *   V: DEVICE n x r row-major, float64, entry (i, j) at V[i * ldv + j].
 *   ldv: leading dimension of V, ldv >= r.
 *   W: DEVICE n x r row-major, float64, entry (i, j) at W[i * ldw + j]; its
 *      rows must not overlap V's (W != V and no aliasing of the two blocks).
 *   ldw: leading dimension of W, ldw >= r.  Columns r .. ld-1 of either
 *      block are neither read nor written.
 *   r: 1 <= r <= 32.
 *   prec: FLP_PREC_FP64, or FLP_PREC_FP32_FILTER (V is rounded to FP32,
 *         the recurrence runs in FP32, W is written in FP64).
 *   format: storage the products read A in: FLP_FORMAT_CSR (A itself),
 *         FLP_FORMAT_SELL (a sliced ELL copy of A, the storage flp_solve uses
 *         by default; the same sums in the same order, so W is bit-identical
 *         to the CSR result) or FLP_FORMAT_AUTO (SELL unless it would store
 *         more than 1.25 times A's nonzeros).  The sliced copy is built on
 *         first use and kept in the calling thread's workspace for later
 *         calls with the same A (the same device arrays and sizes); a caller
 *         that changes A's entries in place between calls releases it first
 *         with flp_release_workspace().  Building it synchronises the stream.
 * Stream-ordered and asynchronous (no host synchronisation unless the
 * workspace must grow, the sliced copy is built, or the launch configuration
 * for this precision, r and matrix size is being tuned; see
 * flp_tune_filter).
 * Errors: FLP_E_ARG (NULL or aliasing blocks, r or ld out of range, bad prec
 *         or format), FLP_E_NOMEM, FLP_E_DEVICE. */
int flp_filter_apply(const flp_filter *p, const flp_csr *A, const double *V, int64_t ldv, double *W,
                     int64_t ldw, int32_t r, int32_t prec, int32_t format, void *stream);

/* flp_filter_apply without device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, allocation-free
 * serving loops, harnesses that forbid hipMalloc).  Same arguments and
 * result as flp_filter_apply with format = FLP_FORMAT_CSR (bit-identical
 * W), except:
 * - the Clenshaw ring buffers (and in FP32 the FP32 copy of V) live in a
 *   fixed 24 MiB device array of the library, one per GPU, held until the
 *   process ends; n * r must not exceed 1048576 (2^20), else FLP_E_NOMEM
 *   before anything is launched;
 * - FLP_PREC_FP32_FILTER needs A->val32 (FLP_E_ARG if NULL);
 * - no tuning: the default launch shape over all r columns.
 * Calls on one GPU share that array, so calls that overlap in time on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  Nothing needs clearing: every step writes its buffer before the
 * next one reads it.  Errors: FLP_E_ARG, FLP_E_NOMEM, FLP_E_DEVICE. */
int flp_filter_apply_noalloc(const flp_filter *p, const flp_csr *A, const double *V, int64_t ldv, double *W,
                             int64_t ldw, int32_t r, int32_t prec, void *stream);

/* Launch configuration of the filter's sparse-matrix step (the Clenshaw
 * step of Section 2.2 as a CSR SpMM over r columns). */
typedef struct flp_tune_info {
    int32_t group_width;   /* columns per filter launch (r / group_width launches per step) */
    int32_t lanes_per_row; /* lanes sharing one matrix row */
    int32_t cols_per_lane; /* consecutive block columns owned by one lane */
    int32_t rows_per_wave; /* matrix rows per 64-lane wavefront (64 / lanes_per_row) */
    int32_t candidates;    /* configurations timed (0: default or forced, not timed) */
    int32_t streaming_loads; /* 1: V and U_{k+2} are read with nontemporal loads */
    double us_per_step;    /* measured microseconds of one step over all r columns (0 if not timed) */
    int32_t tile_chunk;    /* tile-to-XCD mapping: 0 = one contiguous range of row tiles per XCD;
                              c > 0 = chunks of c consecutive row tiles dealt to the 8 XCDs in turn;
                              c < 0 = pencil walk over planes of -c rows: each plane (the rows of one
                              z-plane of a 3D grid in natural order) is cut into 8 column ranges
                              and XCD x takes range x plane after plane, so a row's neighbours in
                              the planes above and below stay in that XCD's L2 */
    int32_t lds_window;    /* 1: each workgroup first copies the rows of the gathered block that it
                              and the 8 rows on either side own into LDS and reads the columns that
                              fall there from LDS (the near-diagonal entries of a banded or stencil
                              matrix), the rest from global memory; same sums.
                              2: sliding window: each workgroup walks one range of consecutive rows
                              (a fraction of a plane of tile_chunk rows, tile_chunk then being that
                              plane length, 0 for none) and keeps the gathered block's rows within
                              window_halo of its current rows in an LDS ring, loading only the rows
                              that enter it at each step; same sums */
    int32_t window_halo;   /* rows on either side of its own that a workgroup reads from LDS
                              (8 for lds_window 1, the tuned halo for 2, else 0) */
} flp_tune_info;

/* Host evaluation of the tile-to-XCD traversal the filter kernels use (the
 * mapping tile_chunk selects): order[b] = the row tile that workgroup b of
 * a launch of `tiles` workgroups processes, rows_per_tile matrix rows per
 * tile (for tile_chunk < 0 the plane holds round(-tile_chunk /
 * rows_per_tile) tiles).  Every mapping is a permutation of [0, tiles).
 * order: HOST int32[tiles].  Host only; needs no device.  Errors: FLP_E_ARG
 * (tiles < 0, rows_per_tile < 1, order NULL). */
int flp_tile_order(int32_t tiles, int32_t tile_chunk, int32_t rows_per_tile, int32_t *order);

/* Autotuner.  The first time a (device, precision, r, storage, size class,
 * plane length) combination is filtered (size class: n to a quarter octave
 * and nonzeros per row to a quarter; plane length: the smallest distance
 * |j - i| >= 1024 from the middle row i to one of its columns j, a 3D
 * grid's N^2), every supported launch shape (rows per wavefront,
 * columns per lane, ordinary or nontemporal loads of the streamed operands),
 * tile-to-XCD mapping (tile_chunk, including the pencil walk over planes of
 * that length) and column-group width is timed on the caller's matrix
 * over a short ring of filter steps and the fastest is kept for the process
 * (timings taken while other work shares the GPU may pick a slower shape,
 * never a different result); the batched
 * and serving engines tune the shape of their segmented launches on the
 * largest active matrix.  All configurations compute every output element
 * with the same operations in the same order, so results are bit-identical.
 * flp_tune_filter runs (or looks up) that tuning for r columns of A read in
 * storage `format` (as flp_filter_apply's) and reports the choice.  A: as
 * for flp_solve (val32 may be NULL).  Synchronises the stream.  Errors:
 * FLP_E_ARG, FLP_E_NOMEM, FLP_E_DEVICE. */
int flp_tune_filter(const flp_csr *A, int32_t r, int32_t prec, int32_t format, void *stream, flp_tune_info *out);

/* The launch shape a filter step runs with, before any tuning: for one
 * solve's kernel (segmented = 0) or the batched engine's segmented kernel
 * (segmented = 1) over a block of r columns (1 <= r <= 32) in precision prec.
 * Fills group_width (= r), lanes_per_row, cols_per_lane and rows_per_wave;
 * lanes_per_row * cols_per_lane >= r always, and where it exceeds r the
 * lanes past column r - 1 have no column and leave the kernel at once.
 * candidates = 0, us_per_step = 0.  Host only; needs no device.
 * Errors: FLP_E_ARG. */
int flp_filter_launch_shape(int32_t r, int32_t prec, int32_t segmented, flp_tune_info *out);

/* on = 1: tune on first use (the default); on = 0: fixed default
 * configuration (16-byte pieces per lane, column groups sized for the
 * 256 MB Infinity Cache). */
void flp_set_autotune(int32_t on);

/* tile_chunk value of flp_set_filter_shape that leaves the mapping to the tuner */
#define FLP_TILE_CHUNK_TUNED INT32_MIN

/* Forces one configuration for every later filter launch (testing and
 * measurement); lanes_per_row = 0, group_width = 0 and tile_chunk =
 * FLP_TILE_CHUNK_TUNED restore tuning.  A shape with no kernel for a given
 * width falls back to the default shape (keeping tile_chunk); a group width
 * that does not divide r is ignored; streaming_loads = 1 reads V and
 * U_{k+2} with nontemporal loads; tile_chunk as in flp_tune_info (any other
 * value than FLP_TILE_CHUNK_TUNED forces it); lds_window = 1 stages the
 * gathered rows near each workgroup's own in LDS, 2 selects the sliding
 * window with its halo and plane found from the matrix's middle row (each
 * solve's own; tile_chunk is then ignored; where no distance beyond 8 rows
 * fits the LDS, the fixed window is used) (flp_tune_info.lds_window;
 * ignored by shapes that do not cover the block in 16-byte pieces). */
void flp_set_filter_shape(int32_t lanes_per_row, int32_t cols_per_lane, int32_t group_width,
                          int32_t streaming_loads, int32_t tile_chunk, int32_t lds_window);

/* Y = A X (plain CSR SpMM, Section 3.2.1).  X, Y: DEVICE n x r row-major
 * with leading dimensions ldx, ldy >= r; 1 <= r <= 32; FP64.  Async. */
int flp_spmm(const flp_csr *A, const double *X, int32_t ldx, double *Y, int32_t ldy,
             int32_t r, void *stream);

/* Full reorthogonalisation of a block against a basis (Section 3.2.2), two
 * passes of classical Gram-Schmidt:
 *   H1 = Q^T W, W -= Q H1, H2 = Q^T W, W -= Q H2, H = H1 + H2.
 *   Q: DEVICE n x k row-major with leading dimension ldq >= k (k >= 1).
 *   W: DEVICE n x r row-major (ld = r), updated in place, 1 <= r <= 16.
 *   H: HOST float64[k * r] row-major (k x r) receiving H1 + H2, or NULL.
 * Synchronises the stream when H is non-NULL. */
int flp_block_orth(const double *Q, int64_t ldq, int32_t k, int32_t n, double *W, int32_t r,
                   double *H, void *stream);

/* Block normalisation W = Qn S (eq. lanczos: S upper triangular with a
 * non-negative diagonal) by Cholesky QR applied twice.
 *   W: DEVICE n x r row-major (ld = r), overwritten by Qn; 1 <= r <= 16.
 *   S: HOST float64[r * r] row-major, receives S.
 * Returns FLP_E_ARG if W is numerically rank deficient.  Synchronous. */
int flp_block_qr(double *W, int32_t n, int32_t r, double *S, void *stream);

/* Estimate [lambda_min, lambda_max] by k0 steps of unfiltered Lanczos with
 * full reorthogonalisation (Section 2.2: a few Lanczos steps), widened by
 * the Ritz residual bounds and 1e-3 of the width, clamped to the Gershgorin
 * enclosure.  Host outputs.  Synchronous. */
int flp_estimate_bounds(const flp_csr *A, int32_t k0, uint64_t seed, double *lmin, double *lmax,
                        void *stream);

/* Every eigenpair of A in [alpha, beta] (program summary; Sections 2-3):
 * bounds (PREPROC) -> filter (Section 2.2) -> block Lanczos on p(A) with
 * full reorthogonalisation (Section 2.3, eq. lanczos) -> periodic
 * convergence checks on the Ritz values of T_k -> Rayleigh-Ritz with A
 * (eq. rayleigh, eq. proj).  opts may be NULL (defaults).  Synchronous.
 * On FLP_OK or FLP_E_NOCONV *out holds a result to free with
 * flp_result_free().  Errors: FLP_E_ARG (also for a filtered solve whose
 * interval, clamped to the bounds, covers all of [lmin, lmax]: the ideal
 * filter is then the constant 1), FLP_E_INTERVAL, FLP_E_NOMEM,
 * FLP_E_NOCONV, FLP_E_DEVICE. */
int flp_solve(const flp_csr *A, double alpha, double beta, const flp_opts *opts,
              flp_result **out);

/* Spectrum slicing on one GPU (Section 5 names slicing as the route to
 * several devices): [alpha, beta] (clamped to the spectrum bounds, which
 * are estimated once unless opts gives them) is cut into nslices
 * sub-intervals of equal width in the angle acos((lambda - c) / e) of the
 * mapped spectrum, so the degree rule gives each slice the same degree;
 * each slice is an independent filtered Lanczos solve on A (seed
 * opts->seed + i * 0x9E3779B97F4A7C15) and all of them advance together as
 * one batch (flp_solve_batch).  The merged result holds every eigenpair in
 * [alpha, beta] in ascending order: slice i contributes its eigenvalues below
 * its upper end (the last slice up to beta), and an eigenpair found by both
 * slices at a boundary (eigenvalues equal to 1e-8 ||A||, eigenvectors
 * overlapping by more than 1/2) is kept once.  stats: work summed over the
 * slices (mv, basis_cols, filter_bytes, t_orth, t_check, t_rr), iters and
 * polish_sweeps the largest slice's, t_mv the shared filter launches' time.
 *   nslices: 1 <= nslices <= 256.
 * Synchronous.  Errors as flp_solve, plus FLP_E_ARG for a bad nslices or an
 * interval too narrow to slice. */
int flp_solve_sliced(const flp_csr *A, double alpha, double beta, int32_t nslices,
                     const flp_opts *opts, flp_result **out);
void flp_result_free(flp_result *res);
/* Copy the result's eigenvectors (count x n doubles, column-major) into the
 * DEVICE buffer dst; stream-ordered (NULL = default stream). */
int flp_result_copy_evecs(const flp_result *res, double *dst, void *stream);

/* Statistics of a batched solve. */
typedef struct flp_batch_stats {
    int32_t solves;           /* problems in the batch */
    int32_t block_steps;      /* lockstep block Lanczos steps */
    int32_t filter_launches;  /* segmented filter launches */
    int32_t graph_captures;   /* HIP graphs captured (one per change of the active set) */
    int32_t graph_replays;    /* block steps replayed from a graph */
    double t_total;           /* seconds: whole call */
    double t_setup;           /* seconds: bounds, filters, start blocks */
    double t_filter;          /* seconds: segmented filter launches (event-timed) */
    double t_orth_check;      /* seconds: Gram-Schmidt, block QR, convergence checks */
    double t_finish;          /* seconds: Rayleigh-Ritz and polish of finished solves */
    double filter_bytes;      /* algorithmic bytes of the segmented filter launches */
    double t_orth;            /* seconds: the segmented Gram-Schmidt and block QR launches
                                 (part of t_orth_check) */
    double orth_bytes;        /* algorithmic bytes of those launches (basis read twice per pass) */
    /* serving only (0 in batched results): */
    int32_t peak_active;      /* most requests in the active set at once */
    int32_t admission_waits;  /* times the next queued request waited for device memory */
    int32_t finish_waits;     /* times a converged request waited for its finish-phase memory */
    double mem_budget;        /* the admission budget in bytes */
    double peak_mem_reserved; /* most device bytes reserved at once (admission + finish phase) */
} flp_batch_stats;

/* Every eigenpair in [alpha[i], beta[i]] of each A[i], for count independent
 * problems solved together (the batched form of flp_solve): one segmented
 * launch per Clenshaw step carries the current filter step of every active
 * solve; solves leave the batch as they converge.
 *   A: HOST array of count pointers to CSR matrices (device data).
 *   alpha, beta: HOST arrays of count doubles.
 *   opts: HOST array of count options or NULL (defaults).  All entries must
 *         have the same block size and precision; opts[0].stream is the
 *         caller's stream (synchronised at entry and exit).
 *   use_graph: 1 to replay each block step's filter launches from a HIP graph.
 *   results: HOST array of count result pointers (filled; free each with
 *            flp_result_free); t_total of each result is its completion time
 *            inside the batch.
 *   codes: HOST array of count per-solve return codes.
 *   stats: optional.
 * Returns FLP_OK if every solve returned FLP_OK or FLP_E_NOCONV, else the
 * first other error.  Synchronous. */
int flp_solve_batch(int32_t count, const flp_csr *const *A, const double *alpha, const double *beta,
                    const flp_opts *opts, int32_t use_graph, flp_result **results, int32_t *codes,
                    flp_batch_stats *stats);

/* ------------------------------------------------------------------ serving
 *
 * A server runs a worker thread that owns the device: requests submitted
 * from any thread are admitted, in submission order, while engine slots and
 * device memory allow, join the active set at the next block-step boundary,
 * share its segmented filter launches, and leave it when they converge
 * (continuous batching).  Device memory is reserved against mem_budget in
 * two parts: at admission, the request's solve buffers (Lanczos basis of
 * max_basis columns, recurrence and block vectors, FP32 and sliced ELL
 * copies; flp_server_footprint); when it converges, its finish phase (the
 * Ritz blocks of the candidate vectors, the result's eigenvectors), before
 * a finisher thread starts it.  A request waits while its part does not fit;
 * one that would run alone is always let through.  Everything is returned
 * when the request completes.
 * While a server runs, other flp_* calls must not use the same device. */
typedef struct flp_server flp_server;

typedef struct flp_server_opts {
    int32_t block;       /* block size of every request (default 8) */
    int32_t prec;        /* precision of every request (default FLP_PREC_FP32_FILTER) */
    int32_t max_active;  /* requests advanced together (default 64) */
    int64_t max_basis;   /* default basis cap per request (default 1024 columns) */
    double mem_budget;   /* device bytes for active requests; <= 0: 70% of free memory */
    int32_t use_graph;   /* replay filter launches from HIP graphs (default 1) */
} flp_server_opts;

void flp_server_opts_default(flp_server_opts *o);
/* Start a server on the current device.  Errors: FLP_E_ARG, FLP_E_DEVICE. */
int flp_server_create(const flp_server_opts *opts, flp_server **out);
/* Queue a request: every eigenpair of A in [alpha, beta].  A's device
 * arrays must stay valid until the result has been retrieved.  opts may be
 * NULL; its block and prec are replaced by the server's.  The server reads
 * A on its own streams only after the work queued on opts->stream (the null
 * stream when opts is NULL or opts->stream is NULL) before this call, so
 * arrays still being written there (a copy, a conversion to FP32) are
 * complete when the request starts.  *ticket names the request.
 * Thread-safe.  Errors: FLP_E_ARG, FLP_E_DEVICE (the event could not be
 * recorded), or the server's device error. */
int flp_server_submit(flp_server *sv, const flp_csr *A, double alpha, double beta, const flp_opts *opts,
                      uint64_t *ticket);
/* FLP_E_PENDING if the request is still queued or running; otherwise its
 * return code (as flp_solve's) with *out set.  result->stats.t_total is the
 * request's latency (submission to completion).  Thread-safe. */
int flp_server_poll(flp_server *sv, uint64_t ticket, flp_result **out);
/* As flp_server_poll, but blocks until the request has finished. */
int flp_server_wait(flp_server *sv, uint64_t ticket, flp_result **out);
/* Cancel a request that has not completed: a queued one is dropped at
 * once, a running one at its next block-step boundary (its device memory
 * returns to the admission budget); flp_server_poll/wait then return
 * FLP_E_CANCELLED with *out = NULL.  A request whose result is already
 * ready, or being assembled, is not affected.  Thread-safe.  Errors:
 * FLP_E_ARG (unknown ticket). */
int flp_server_cancel(flp_server *sv, uint64_t ticket);
/* Engine statistics so far (solves = requests submitted). */
int flp_server_stats(flp_server *sv, flp_batch_stats *out);
/* Device bytes a request for A with options opts (NULL: defaults; block,
 * precision and the basis cap as flp_server_submit sets them) reserves at
 * admission.  Host only.  Errors: FLP_E_ARG. */
int flp_server_footprint(const flp_server *sv, const flp_csr *A, const flp_opts *opts, double *bytes);
/* Finish every queued request, stop the worker, free unretrieved results. */
int flp_server_destroy(flp_server *sv);

/* Dense symmetric eigensolver used for the projected problems (Section
 * 3.2.2 solves T_k's eigenproblem on the CPU with a banded symmetric
 * eigensolver).  Host only; no GPU needed.
 *   M: HOST float64[N * N] row-major symmetric with semi-bandwidth bw
 *      (bw = N - 1 for dense), not modified.
 *   evals: HOST float64[N], ascending.
 *   evecs: HOST float64[N * N] row-major (column j = eigenvector j), or NULL.
 * Returns FLP_OK or FLP_E_ARG. */
int flp_host_sym_eig(int32_t N, int32_t bw, const double *M, double *evals, double *evecs);

/* Free the calling thread's workspace on the current device. */
void flp_release_workspace(void);

/* Device memory.  By default the library allocates with hipMalloc and frees
 * with hipFree.  flp_set_allocator routes every later device allocation
 * (workspace, solve buffers, result eigenvectors) through alloc/free instead
 * (for example a framework's caching allocator); alloc returns NULL on
 * failure (reported as FLP_E_NOMEM).  Memory always goes back to the pair
 * that allocated it, and the device is synchronised before it is handed to
 * a caller's free function.  NULL, NULL restores hipMalloc/hipFree.  Change
 * the setting while no call is running; the functions may be called from
 * the library's own threads (server worker, finishers). */
typedef void *(*flp_alloc_fn)(size_t bytes, void *ctx);
typedef void (*flp_free_fn)(void *ptr, void *ctx);
void flp_set_allocator(flp_alloc_fn alloc, flp_free_fn free_fn, void *ctx);

/* Opt-in symmetry check, O(nnz) on the device (the library assumes
 * A = A^T with both triangles stored, Section 3.2.1): every stored a_ij
 * needs a stored a_ji with |a_ij - a_ji| <= tol * max(|a_ij|, |a_ji|)
 * (tol >= 0; 0 asks for equality).  Synchronous.  Returns FLP_OK, or
 * FLP_E_NOTSYM with the number of failing entries in flp_last_error(), or
 * FLP_E_ARG / FLP_E_DEVICE. */
int flp_check_symmetric(const flp_csr *A, double tol, void *stream);

/* Message of the last failing call on this thread ("" if none). */
const char *flp_last_error(void);

/* Library version string. */
const char *flp_version(void);

/* Sizes in bytes of the ABI structs, for bindings to check their mirrors:
 * writes up to cap values to sizes[] in the order flp_csr, flp_opts,
 * flp_stats, flp_result, flp_tune_info, flp_batch_stats, flp_server_opts
 * and returns how many there are (7).  Host only; needs no device. */
int32_t flp_abi_sizes(int64_t *sizes, int32_t cap);

#ifdef __cplusplus
}
#endif

#endif /* FLP_H */
