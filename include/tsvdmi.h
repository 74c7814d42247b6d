/*
 * tsvdmi: cosine-transform t-SVD, t-SVT and TNN-C tensor completion on one
 * AMD Instinct MI355X (gfx950).
 *
 * The operations follow Xu, Zhao and Ng, "A Fast Algorithm for Cosine
 * Transform Based Tensor Singular Value Decomposition" (arXiv 1902.03070):
 *   - Section 3: the transform along tubes, Xbar = dct(X,[],3), read as the
 *     orthonormal DCT-II C[k][t] = s_k cos(pi (2t+1) k / (2 n3)).
 *   - Equation (tproduct dct): the DCT t-product, Zbar^(k) = Xbar^(k) Ybar^(k).
 *   - Theorem 4: the DCT t-SVD, computed as the SVD of every frontal slice of
 *     Xbar.
 *   - Theorem 5 with Algorithm 1: tensor singular value thresholding.
 *   - Algorithm 1: ADMM for the TNN-C completion model.
 *
 * Conventions for every entry point
 *   - Tensors are real n1 x n2 x n3, column-major with contiguous frontal
 *     slices: element (i,j,k) is at index i + n1*j + n1*n2*k (0-based).
 *   - Tensor pointers are DEVICE pointers to caller-owned memory on the
 *     context's device.  The element type is double for TSVD_FP64 and float
 *     for TSVD_FP32 and TSVD_MIXED.  The library never frees caller memory.
 *     Inputs and outputs must not overlap unless stated.
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  Work is
 *     enqueued on it and the call returns without waiting, except where a
 *     call says it synchronizes.
 *   - A context owns its device workspace, the DCT matrices, captured graphs
 *     and tuning results.  One context per host thread, or external locking.
 *   - Tube length n3 (the transform along the tubes): n3 <= 128 runs on the
 *     matrix cores; 128 < n3 <= 512 (DCT and Fourier paths) on the fast
 *     O(n3 log n3) transform (Makhoul's reordering, Bluestein's chirp,
 *     radix-8/16 FFTs) in FP64 arithmetic for double data and FP32 for float
 *     data; other tubes longer than 128 (caller-
 *     given transforms, tsvt_dct_noalloc, n3 > 512) on the dense vector-ALU
 *     kernel, which holds at most 304 (double data) or 608 (float data):
 *     beyond that a call returns TSVD_EINVAL.
 *   - Return value: TSVD_OK, a positive warning (outputs written), or a
 *     negative error (outputs undefined).  Errors found on the device
 *     (non-finite input, Jacobi not converged, a wait that timed out) are
 *     recorded in the context and returned by tsvd_sync_status, or directly
 *     by a call that synchronizes.  No C++ exception crosses this interface.
 */
#ifndef TSVDMI_H
#define TSVDMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tsvd_ctx tsvd_ctx;

/* Precision of a call.
 *   TSVD_FP64  : double data; every step in FP64.
 *   TSVD_FP32  : float data; transforms on FP32 matrix cores; Jacobi sweeps in
 *                FP32 with the rotation angle and the orthogonality test in
 *                FP64.
 *   TSVD_MIXED : float data; transforms on BF16 matrix cores with a hi+lo
 *                split (three products, FP32 accumulation); Jacobi sweeps in
 *                FP32 with FP64 angles and test, then one final sweep whose
 *                dot products and angles are computed in FP64 (its
 *                rotations act on the FP32 values in FP32). */
enum { TSVD_FP64 = 0, TSVD_FP32 = 1, TSVD_MIXED = 2 };

enum {
    TSVD_OK = 0,
    TSVD_WARN_NOCONV = 1,  /* a Jacobi SVD hit the sweep limit; outputs written */
    TSVD_EINVAL = -1,      /* bad argument: size <= 0, tau < 0, beta <= 0, NULL, unknown precision */
    TSVD_ENOMEM = -2,      /* device allocation failed */
    TSVD_EHIP = -3,        /* a HIP runtime call failed (see tsvd_last_error) */
    TSVD_ENONFINITE = -4,  /* the input holds a NaN or an infinity */
    TSVD_EBUSY = -5,       /* admission refused: request exceeds the memory budget */
    TSVD_ETIMEOUT = -6,    /* a bounded device wait or a host deadline expired */
    TSVD_ECANCELED = -7    /* a serving request was cancelled */
};

/* Context.  `device` is a HIP device ordinal.  Returns TSVD_OK and sets *ctx. */
int tsvd_create(tsvd_ctx** ctx, int device);
void tsvd_destroy(tsvd_ctx* ctx);
/* Message of the last failure on this context (never NULL). */
const char* tsvd_last_error(const tsvd_ctx* ctx);

/* Options (set before use; values are doubles for a uniform interface). */
enum {
    TSVD_OPT_MAX_SWEEPS = 0,   /* Jacobi sweep limit, 1..63 (default 30); with TSVD_OPT_KEPT_COLUMNS
                                  the kept-column iteration and the full iteration it may fall
                                  back to each have this limit */
    TSVD_OPT_SYNC_STATUS = 1,  /* 1: each call synchronizes and returns device status (default);
                                  0: calls are asynchronous, status via tsvd_sync_status */
    TSVD_OPT_TEAM_SIZE = 2,    /* 0: automatic; >0: workgroups per frontal slice in the Jacobi
                                  kernel for slices too large for one workgroup's LDS */
    TSVD_OPT_SPIN_LIMIT = 3,   /* polls before a device wait gives up (test hook; default 2^24) */
    TSVD_OPT_PROFILE = 4,      /* 1: record HIP events around every kernel phase on the launch
                                  stream (read with tsvd_get_stats); 2: only around the Jacobi
                                  launches (phase 1; each event pair costs a few microseconds
                                  of GPU time); 0: off (default) */
    TSVD_OPT_GRAPHS = 5,       /* 1: complete_tensor replays one captured iteration as a HIP graph
                                  (default; not while profiling); 0: direct launches */
    TSVD_OPT_AUTOTUNE = 6,     /* 1: choose Jacobi tiles by timing the candidates (default); 0: the
                                  built-in heuristic.  See tsvd_get_tile. */
    TSVD_OPT_GROUP_LANES = 7,  /* 0: automatic; 16, 32 or 64: lanes per column-pair group in the
                                  Jacobi kernels (64: multi-workgroup kernel only, one column pair
                                  per wavefront; a forced setting, like TEAM_SIZE, disables tuning) */
    TSVD_OPT_GROUP_COLUMNS = 8, /* 0: automatic; 1 or 2: columns each lane group of the multi-workgroup
                                  Jacobi kernel holds (2: two independent rotations at a time; not
                                  with V).  A forced setting disables tuning. */
    TSVD_OPT_WARM_START = 9,   /* complete_tensor: -1 (default) warm-start each iteration's Jacobi SVDs
                                  from the previous iteration's right singular vectors, resetting
                                  them to the identity every 64 iterations; N >= 1: reset every N
                                  iterations; 0: cold starts */
    TSVD_OPT_COOPERATIVE = 10, /* 0 (default): ordinary launches of the multi-workgroup Jacobi kernel
                                  (its grid is sized so that every team is resident, and a team
                                  wait that exceeds the spin limit returns TSVD_ETIMEOUT); 1:
                                  cooperative launches outside graph capture (the runtime then
                                  refuses a grid that cannot be resident).  Both run at the same
                                  speed; a process that made cooperative launches ended in a
                                  segmentation fault at exit under rocprofv3, one that made only
                                  ordinary launches did not.  The environment variable
                                  TSVDMI_COOPERATIVE=1 sets 1 at context creation. */
    TSVD_OPT_GRAM = 11,        /* block-Gram Jacobi kernel for slices that need several workgroups
                                  (column blocks of 16: Gram matrices and the accumulated rotations
                                  applied on the matrix cores): 0 a candidate of the tuner, 1
                                  forced (team size from TSVD_OPT_TEAM_SIZE, else one workgroup
                                  per 32 columns), -1 (default) never used */
    TSVD_OPT_LONG_TUBES = 12,  /* DCT tubes of 129..512: 0 (default) the fast O(n3 log n3)
                                  transform, 1 the dense vector-ALU product where its LDS tile
                                  fits (n3 <= 304 for double data, 608 for float) */
    TSVD_OPT_TEAM_SLOTS = 13,  /* 0: automatic; N > 0: at most N slices in flight per XCD in the
                                  multi-workgroup Jacobi kernel (teams then take several slices
                                  in turn; the tuner also tries the count whose A and V fit an
                                  XCD's L2).  A forced setting, like TEAM_SIZE, disables tuning. */
    TSVD_OPT_KEPT_COLUMNS = 14 /* tsvt_dct, tsvt_transform, tsvt_dft (tau > 0) and complete_tensor
                                  without the warm start (TSVD_OPT_WARM_START 0), when the
                                  multi-workgroup Jacobi kernel with one column per lane group
                                  runs the SVDs: 1 (default) each slice's iteration evaluates
                                  only the column pairs that touch a column of norm > tau and
                                  stops once those columns are orthogonal to all others
                                  (Theorem 5 needs no more); the slice is then certified (the
                                  remaining columns of spectral norm <= tau) or run through the
                                  full iteration.  A slice whose kept set is large or settles
                                  slowly (no gap below tau) turns into the full iteration after
                                  its second or third sweep.  0: the full iteration for every
                                  slice.  tsvd_stats counts the pairs evaluated and the slices
                                  the certificate rejected. */
};
int tsvd_set_option(tsvd_ctx* ctx, int option, double value);
double tsvd_get_option(const tsvd_ctx* ctx, int option);

/* Wait for `stream`, then return and clear the device status accumulated by
 * asynchronous calls on this context (TSVD_OK, TSVD_WARN_NOCONV,
 * TSVD_ENONFINITE or TSVD_ETIMEOUT).  *max_sweeps_out (may be NULL) gets the
 * largest Jacobi sweep count seen. */
int tsvd_sync_status(tsvd_ctx* ctx, void* stream, int* max_sweeps_out);

/* Jacobi tile of a tensor shape (the one the next call with this shape uses).
 * A slice of a t-SVT is the tall m x p matrix, m = max(n1,n2), p = min(n1,n2)
 * (Theorem 4 takes one SVD per transformed frontal slice); its column pairs
 * are handled by groups of G lanes, either with the whole slice resident in
 * one workgroup's LDS or by a team of W workgroups exchanging column blocks.
 * With TSVD_OPT_AUTOTUNE on and no forced option, the first request for a
 * shape class times every candidate tile on synthetic slices of that shape on
 * the context's own stream (synchronizing the device and allocating a
 * temporary buffer) and caches the fastest for the process; the class is
 * (precision, m, p, n3, with_v), or (precision, m, p, with_v) for batched
 * calls (batched != 0).  If the environment variable TSVDMI_TILE_CACHE names
 * a file, tuned tiles are read from and appended to it; if TSVDMI_TUNE_LOG is
 * set, every candidate's time (or -1 when it failed) goes to stderr.  No tuning happens
 * while `stream` of a call is being captured.  Results of different tiles
 * agree to the precision's tolerance, not bitwise.
 * out[6]: team (0 resident, 1 team), G, W (0 when resident), workgroup size,
 * source (0 heuristic, 1 autotuned, 2 forced by options), columns per lane
 * group (0 when resident). */
int tsvd_get_tile(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, int batched, int with_v,
                  int32_t* out);

/* Counters since the last reset.  Phases: 0 forward transform (with the
 * completion prologue), 1 Jacobi SVD, 2 thresholding and rebuild, 3 inverse
 * transform (with the completion epilogue), 4 warm start of the completion's
 * Jacobi (reset of V and the product Zbar V), 5 threshold certificate of the
 * kept-column mode (TSVD_OPT_KEPT_COLUMNS) with the full iteration of the
 * slices it rejects.  ms/launches are filled only while TSVD_OPT_PROFILE is 1
 * (event pairs on the launch stream).  Always counted: slice_sweeps, Jacobi
 * sweeps summed over all slices processed; pairs, column pairs evaluated by
 * the kept-column mode; fallback_slices, slices its certificate rejected.
 * Synchronizes `stream`. */
typedef struct {
    int64_t slice_sweeps;
    double ms[6];
    int64_t launches[6];
    int64_t pairs;
    int64_t fallback_slices;
} tsvd_stats;
int tsvd_get_stats(tsvd_ctx* ctx, void* stream, tsvd_stats* out, int reset);

/* DCT t-product, equation (tproduct dct):  Z = X * Y, i.e.
 * Zbar^(k) = Xbar^(k) Ybar^(k) for every k, with Xbar = dct(X,[],3).
 * X: n1 x n2 x n3, Y: n2 x n4 x n3, Z: n1 x n4 x n3 (Z must not alias X, Y). */
int tprod_dct(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n4, int64_t n3, const void* X,
              const void* Y, void* Z, void* stream);

/* DCT t-SVD, Theorem 4, thin form with p = min(n1,n2):
 *   U: n1 x p x n3, S: p x n3 (column k holds the singular values of the
 *   transformed slice k, descending), V: n2 x p x n3.
 * Flag TSVD_FULL: the full factors of Theorem 4, U: n1 x n1 x n3 and
 * V: n2 x n2 x n3, orthogonal in every transformed slice (S stays p x n3, the
 * diagonal of the f-diagonal n1 x n2 x n3 tensor).  The first p columns are
 * the thin ones; each of the longer side's other columns is the standard
 * basis vector with the largest part outside the span of the columns before
 * it (first on ties), projected out twice (Gram-Schmidt), normalized, largest
 * entry positive.  A zero singular value's left vector is completed the same
 * way (with the sign convention of its pair), in both forms.
 * Default: spatial-domain factors, so that X = U * S * V^T with the library's
 * tprod_dct (S expanded to the f-diagonal p x p x n3 tensor whose tubes are
 * idct of the rows of S: S itself is returned in the spatial domain).  Flag
 * TSVD_TRANSFORM_DOMAIN returns Ubar, the singular values sigma and Vbar
 * instead.  Sign convention: in
 * each transformed slice, the largest-magnitude entry of every left singular
 * vector is positive.  U or V may be NULL when not wanted. */
enum { TSVD_TRANSFORM_DOMAIN = 1, TSVD_FULL = 2 };
int tsvd_dct(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const void* X, void* U, void* S,
             void* V, int flags, void* stream);

/* Tensor singular value thresholding, Theorem 5 and Algorithm 1's loop body:
 * Y = idct_k( Ubar^(k) (Sbar^(k) - tau)_+ Vbar^(k)^T ) where
 * Zbar^(k) = Ubar^(k) Sbar^(k) Vbar^(k)^T.  Threshold `tau` (>= 0) is applied
 * to the singular values of the orthonormal-DCT slices.
 * ranks_out: NULL or a HOST array of n3 int32 that receives #{sigma > tau}
 * per slice; when given, the call synchronizes.  Y may alias Z. */
int tsvt_dct(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const void* Z, void* Y, double tau,
             int32_t* ranks_out, void* stream);

/* tsvt_dct for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, result and status as tsvt_dct (to the precision's tolerance:
 * the Jacobi tile is the one tsvt_dct has tuned for this shape in this
 * process, else the default one, since tuning needs memory).  Every device
 * buffer of the call - workspace, transform matrices (built on the device) -
 * lives in one fixed array of TSVD_NOALLOC_MAX_BYTES compiled into the
 * library, one per GPU, held until the process ends; the control block is the
 * one tsvd_create allocated.  The call makes no device allocation and no
 * profiling events.
 *   - A tensor whose workspace does not fit returns TSVD_EINVAL (the message
 *     gives the bytes needed); 256 x 256 x 31 fits in every precision.
 *   - All calls on one GPU share that GPU's array, which keeps the last call's
 *     contents: calls that overlap on one GPU (two streams, two threads, two
 *     contexts) race and give undefined results.  Order them. */
#define TSVD_NOALLOC_MAX_BYTES ((size_t)128 << 20)
int tsvt_dct_noalloc(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const void* Z, void* Y,
                     double tau, int32_t* ranks_out, void* stream);

/* t-SVT under another invertible transform along the tubes (concluding
 * remarks: transforms other than the DCT in the t-SVD framework):
 *   Zbar(:,:,k) = sum_t L[k][t] Z(:,:,t);  Ybar^(k) = Ubar (Sbar - tau)_+ Vbar^T
 *   of Zbar^(k);  Y(:,:,t) = sum_k Linv[t][k] Ybar(:,:,k).
 * L: HOST row-major n3 x n3 FP64 matrix, invertible; Linv is computed on the
 * host in FP64 (Gauss-Jordan with partial pivoting).  With L = the
 * orthonormal DCT-II matrix this is tsvt_dct.  For an orthogonal L the result
 * is the proximal map of tau * sum_k ||(L Y)^(k)||_*.  L is copied; its device
 * form is kept in the context and rebuilt when L changes (which waits for the
 * stream).  TSVD_EINVAL for a NULL, singular or non-finite L; otherwise as
 * tsvt_dct. */
int tsvt_transform(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const double* L, const void* Z,
                   void* Y, double tau, int32_t* ranks_out, void* stream);

/* t-SVT in the Fourier domain (Section 2: the DFT-based t-SVD, TNN-F): every
 * frontal slice of the unnormalized Zt = fft(Z,[],3) is thresholded at tau,
 * Yt^(k) = U (S - tau)_+ V^H, and Y = ifft(Yt,[],3), real for real Z.  This is
 * the proximal map of tau * TNN-F (the 1/n3 of TNN-F cancels the unnormalized
 * transform's scale).  Conjugate symmetry leaves floor((n3-1)/2) complex
 * slices and one or two real ones; a complex slice B + iC is thresholded
 * through its real form [[B, -C], [C, B]] (same singular values, each twice)
 * on the DCT path's kernels.  ranks_out (host, n3 entries or NULL) gets the
 * rank of every Fourier slice k = 0..n3-1.  Slices of at most 256 rows and
 * columns (their real forms are at most 512).  Otherwise as tsvt_dct. */
int tsvt_dft(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const void* Z, void* Y, double tau,
             int32_t* ranks_out, void* stream);

/* TNN-C, equation (equTNN1): (1/n3) sum_k ||Xbar^(k)||_*, with Xbar =
 * dct(X,[],3).  *out receives the value (host); the call synchronizes. */
int tnn_c(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const void* X, double* out, void* stream);

/* TNN-F, equation (tnn): (1/n3) sum_k ||Xt^(k)||_* over the slices of the
 * unnormalized Xt = fft(X,[],3) (same slice limit as tsvt_dft).  *out
 * receives the value (host); the call synchronizes. */
int tnn_f(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const void* X, double* out, void* stream);

/* Algorithm 1 (ADMM for TNN-C completion).
 *   B    : observed data (only entries with mask != 0 are read).
 *   mask : DEVICE uint8 array, N = n1*n2*n3 entries, nonzero = observed.
 *   X    : in = initial iterate, out = the recovered tensor.  With
 *          opts->init_observed = 1 the input contents are ignored and the
 *          library starts from Algorithm 1's initial iterate, B on the
 *          observed set and 0 elsewhere (formed on the device).
 * Iteration l of the call uses beta_l = opts->beta, or
 * 1/opts->tau_schedule[start_iter + l] when a schedule is given, in Z = X - M/beta_l, in
 * the X-update and in the multiplier update, and thresholds at
 * tau_l = 1/beta_l.  It stops after max_iter iterations, or earlier when the
 * relative change ||X_new - X||_F / ||X||_F <= tol (tested every check_every
 * iterations; tol <= 0 disables the test).  M_init (DEVICE, may be NULL for
 * zero) and M_out (DEVICE, may be NULL) carry the multiplier for warm starts.
 * The whole iteration runs on the device and is replayed as a captured HIP
 * graph; the call synchronizes.  Every iteration checks its input
 * Z = X - M/beta_l for NaN and infinity: the call then returns
 * TSVD_ENONFINITE.  Any max_iter > 0 is accepted (the device keeps the last
 * 4096 relative changes in a ring). */
typedef struct {
    int max_iter;               /* L (> 0) */
    double tol;                 /* stopping tolerance on the relative change */
    double beta;                /* fixed penalty when tau_schedule is NULL (> 0) */
    const double* tau_schedule; /* HOST array of thresholds (> 0), or NULL; this call's
                                   iteration i uses tau_schedule[start_iter + i] */
    int check_every;            /* iterations between host checks of tol (>= 1) */
    int start_iter;             /* schedule offset for warm starts; 0 normally */
    const void* M_init;
    void* M_out;
    int init_observed;          /* 1: start from X = B on the observed set, 0 elsewhere */
} tsvd_complete_opts;
typedef struct {
    int iters;         /* iterations run */
    double rel_change; /* last relative change */
    int status;        /* TSVD_OK or TSVD_WARN_NOCONV */
    int max_sweeps;    /* largest Jacobi sweep count seen */
} tsvd_complete_info;
int complete_tensor(tsvd_ctx* ctx, int prec, int64_t n1, int64_t n2, int64_t n3, const void* B,
                    const uint8_t* mask, void* X, const tsvd_complete_opts* opts, tsvd_complete_info* info,
                    void* stream);

/* Batched t-SVT (Theorem 5 per tensor) of `count` tensors of independent
 * shapes.  The Jacobi step of all tensors is one persistent launch per row
 * geometry present (at most 8; usually 1 or 2), each draining a device work
 * list of (tensor, slice) tasks, largest first.  dims: HOST array of 3*count
 * sizes (n1,n2,n3 per tensor); Z, Y: HOST arrays of DEVICE pointers; tau:
 * HOST array of thresholds.  A tensor's tile depends only on its own shape
 * and each task is done by one workgroup, so its result is bitwise the same
 * as in a batched call holding it alone; it agrees with tsvt_dct on it to the
 * precision's tolerance (tsvt_dct may use a multi-workgroup team).
 * status_out: NULL, or a HOST array of `count` codes.  When given, the call
 * synchronizes and writes every tensor's own status (TSVD_OK,
 * TSVD_WARN_NOCONV, TSVD_ENONFINITE or TSVD_ETIMEOUT), so that one bad
 * tensor does not mark the others; the return value then reports only
 * argument and launch errors.  When NULL, the statuses of all tensors are
 * accumulated as for any asynchronous call. */
int tsvt_dct_batched(tsvd_ctx* ctx, int prec, int count, const int64_t* dims, const void* const* Z,
                     void* const* Y, const double* tau, int32_t* status_out, void* stream);

/* ---------------------------------------------------------------------------
 * Serving: a host thread that admits t-SVT and completion requests by device
 * memory footprint, keeps every admitted request's iterates on the device, and
 * advances all admitted requests together, one batched step per tick
 * (continuous batching: a request that arrives while others run joins at the
 * next tick; a finished one leaves and frees its memory).
 * ------------------------------------------------------------------------- */
typedef struct tsvd_server tsvd_server;
enum { TSVD_REQ_TSVT = 0, TSVD_REQ_COMPLETE = 1 };
typedef struct {
    int kind;              /* TSVD_REQ_TSVT or TSVD_REQ_COMPLETE */
    int64_t n1, n2, n3;
    const float* input;    /* HOST: Z (t-SVT) or B (completion), n1*n2*n3 floats, copied at submit */
    const uint8_t* mask;   /* HOST: completion observed set, copied at submit; NULL for t-SVT */
    double tau;            /* t-SVT threshold */
    int iters;             /* completion: iterations, tau decays geometrically tau0 -> tau1 */
    double tau0, tau1;
    double deadline_s;     /* > 0: the request ends with TSVD_ETIMEOUT unless done this many seconds
                              after submit (checked between ticks); <= 0: no deadline */
} tsvd_request;
/* budget_bytes: device memory the server may hold for admitted requests;
 * max_active: most requests advanced per tick.  With FP32 or MIXED data a
 * completion request warm-starts its Jacobi SVDs from its previous
 * iteration's right singular vectors, kept on the device, following the
 * context's TSVD_OPT_WARM_START (read at creation). */
int tsvd_server_create(tsvd_server** srv, tsvd_ctx* ctx, int prec, int64_t budget_bytes, int max_active);
/* Copies the request; returns a request id > 0, TSVD_EBUSY when it can never
 * fit the budget, or TSVD_EINVAL for bad sizes or parameters or a shape the
 * batched kernels cannot hold (frontal slices above 512 rows or columns).
 * Admission is first in, first out: a queued request is never overtaken. */
int64_t tsvd_server_submit(tsvd_server* srv, const tsvd_request* req);
/* Cancels request `id`: a queued one ends at once, a running one before its
 * next step; either then polls as TSVD_ECANCELED.  Returns 0, 1 if it had
 * already ended, or TSVD_EINVAL for an unknown id. */
int tsvd_server_cancel(tsvd_server* srv, int64_t id);
/* Non-blocking poll.  When request `id` is done, fills `out` (HOST, n1*n2*n3
 * floats) and the times (seconds on the server's steady clock) and returns 1
 * (2 when one of its Jacobi SVDs hit the sweep limit); 0 if not done yet; its
 * negative status if it failed (only that request: TSVD_ENONFINITE,
 * TSVD_ETIMEOUT, TSVD_ECANCELED, ...), or TSVD_EINVAL for an unknown id.  A
 * done request is forgotten after it is polled. */
int tsvd_server_poll(tsvd_server* srv, int64_t id, float* out, double* t_submit, double* t_admit, double* t_done);
/* Server clock now (seconds). */
double tsvd_server_now(tsvd_server* srv);
/* Statistics: admitted, completed, ticks, peak bytes held. */
int tsvd_server_stats(tsvd_server* srv, int64_t* admitted, int64_t* completed, int64_t* ticks, int64_t* peak_bytes);
void tsvd_server_destroy(tsvd_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* TSVDMI_H */
