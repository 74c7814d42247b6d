// Declarations of the Jacobi SVD kernels (jacobi.hip) and the constants and
// control structures they share with the rest of libtsvdmi.  Not part of the
// public interface (include/tsvdmi.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tsvd {

constexpr int kMaxSweeps = 64;       // hard cap on Jacobi sweeps (per-sweep counters are sized by it)
constexpr int kRotStride = 4 * kMaxSweeps;  // per slice: rotations per sweep, large-angle pairs per sweep, then
                                            // (kept-column mode) pairs evaluated and pairs with cosine > 1e-2
constexpr int kKeepMaxSweeps = 16;   // kept-column sweeps before a slice that has not converged turns into
                                     // the full iteration
constexpr int kWave = 64;            // CDNA wavefront width
constexpr int kMaxEpl = 8;           // rows per lane in the Jacobi kernels: m <= 512
constexpr int kMaxRows = kWave * kMaxEpl;
constexpr int kTeamMaxThreads = 512;  // launch bound of the Jacobi team kernel
constexpr int kTeamMaxThreads64 = 1024;  // ... with 64-lane groups (one column pair per wavefront)
constexpr int kLdsPad = 16;            // extra elements per LDS column (spreads lane groups over banks)
constexpr int kNormSlots = 16;       // slot pairs of the completion's change norms (256 bytes)
constexpr int kLdsBudget = 160 * 1024 - 8 * 1024;  // dynamic LDS per workgroup (gfx950: 160 KB, minus static use)

// Device status bits (accumulated with atomicOr in ctrl->status).
enum : int { kStNonFinite = 1, kStNoConv = 2, kStTimeout = 4 };

// Per-launch control block in device memory.
struct Ctrl {
    int status;      // kSt* bits
    int max_sweeps;  // largest sweep count seen (atomicMax)
    int iter;        // completion iteration counter (graph-captured loops)
    int fallback;    // slices the threshold certificate sent back to a full Jacobi SVD (statistics)
    unsigned long long slice_sweeps;  // sweeps executed, summed over slices (statistics)
    unsigned long long pairs;         // column pairs evaluated in the kept-column mode (statistics)
};

// One Jacobi problem set: all frontal slices of one tensor, in "tall" form.
// Slice k's tall matrix T_k (m x p, m >= p) is, element (r, c):
//   src[k*src_ss + r*src_rs + c*src_cs]
// i.e. the transformed slice itself (n1 >= n2) or its transpose.
struct JacobiJob {
    const void* src;   // transformed tensor Zbar (n1 x n2 x n3)
    void* A;           // work/output: m x p per slice, ld = m, slice stride m*p
    void* V;           // p x p per slice (ld = p) or nullptr
    int* rot;          // [n3 * kRotStride] per-sweep counters (zeroed before launch): rotations, then
                       // pairs whose cosine exceeded sqrt(skip2)
    int* sweeps;       // [n3] sweeps used per slice (-1 = not converged)
    int64_t src_ss, src_rs, src_cs;
    int m, p, n3;
    int G;             // lanes per column pair (16 or 32)
    int R;             // rows per lane (4, 8, 12 or 16): R*G >= m
    int ldv;           // LDS leading dimension of V columns (multiple of G, >= p)
    int b;             // block width for the team kernel (even)
    int nb;            // number of column blocks (even) = ceil(p / b) rounded up to even
    int refine64;      // 1: after convergence run one sweep with FP64 arithmetic (FP32 data)
    int vinit;         // with V: 1 starts V from the contents of V (a warm start), 0 from the identity
    double tol;        // rotate a pair iff |x.y| > tol |x| |y| (precision dependent, set on the host)
    double skip2;      // a sweep whose pairs all have (x.y)^2 <= skip2 |x|^2 |y|^2 ends the iteration
                       // (the next sweep would rotate by angles far below tol: no check sweep)
    Ctrl* ctrl;        // per-job status and counters (batched steps), or nullptr: the launch's block
    // Kept-column mode (team kernel with one column per lane group): only
    // the pairs with a column of squared norm above keep2 (tau^2 of a t-SVT)
    // are evaluated and count towards convergence; a pair of two columns at or
    // below it (a "rest" pair) is skipped.  The iteration ends once the columns
    // above the threshold are orthogonal to all others -- all a singular value
    // thresholding needs, provided the remaining columns have spectral norm
    // <= tau, which the threshold certificate checks afterwards (a slice that
    // fails goes through the full iteration).  One last sweep on the kept pairs
    // (FP64 arithmetic for the mixed path) follows convergence.  The kept
    // columns settle fast when the singular values have a gap below tau and
    // slowly when they do not, so the slice turns into the full iteration for
    // good after a sweep (past the first) that evaluated over 40% of all pairs,
    // after a sweep with an unchanged kept set in which the pairs with cosine
    // > 1e-2 fell by less than a factor 0.5 (or two in a row by less than
    // 0.35), or after kKeepMaxSweeps sweeps; a slice that converges that way is
    // marked in full[] (it needs no certificate).  A slice that does not converge in this
    // mode is not flagged TSVD_WARN_NOCONV here: the certificate sends it back.
    int keep;          // 0: every pair, to full convergence; 1: kept-column mode
    double keep2;      // the mode's squared threshold (> 0), or
    const double* keep_sched;  // (device) thresholds by iteration: tau = keep_sched[ctrl->iter]
    int* full;         // [n3] (kept-column mode) set to 1 for a slice that converged as the full iteration
    const int* skip;   // [n3] or nullptr: nonzero = the slice is done, the launch leaves it untouched
};

struct TeamSched {
    int W;             // workgroups per team
    int nwg;           // workgroups in the grid (a multiple of 8 W: whole teams on each XCD)
    int* ctl;          // team formation and barrier counters, kTeamCtlInts + nwg (1 + nb) ints, zeroed
};
constexpr int kTeamCtlInts = 32;
constexpr int kJobCtrlBytes = 256;  // per-job control block of a batched step (a Ctrl, padded)

// Jacobi one-sided SVD of every slice.  Single tensor: `job1` by value, task
// t = slice t (jobs_dev == nullptr).  Batched: job table and task list in
// device memory.
hipError_t launch_jacobi_resident(int prec, const JacobiJob& job1, const JacobiJob* jobs_dev, const int* task_job,
                                  const int* task_slice, int ntasks, int max_sweeps, Ctrl* ctrl, int lds_bytes,
                                  int threads, int with_v, hipStream_t s);
// K: lane-group columns (1, or 2 with two I columns per group and no V; the
// block width job.b is then 2 * threads / G).
hipError_t launch_jacobi_team(int prec, const JacobiJob& job, int ntasks, const TeamSched& ts, int max_sweeps,
                              Ctrl* ctrl, int lds_bytes, int threads, int with_v, int spin_limit, int R, int G, int K,
                              int coop, hipStream_t s);
// Block-Gram multi-workgroup kernel (blocks of 16 columns, 256 threads per
// workgroup, matrix-core Gram matrices and updates); job.b must be 16.
// With V and job.vinit == 0 it first sets V to the identity.
hipError_t launch_jacobi_gram(int prec, const JacobiJob& job, int ntasks, const TeamSched& ts, int max_sweeps,
                              Ctrl* ctrl, int with_v, int spin_limit, int coop, hipStream_t s);
int jacobi_gram_lds_bytes(int prec, int m);
constexpr int kGramBlock = 16;  // columns per block of the block-Gram kernel
int jacobi_gram_max_resident(int prec, int m, int with_v);
// One persistent launch over (tensor, slice) tasks drawn from *queue (zeroed).
// One persistent launch per row geometry (R, G) present in the batch.
hipError_t launch_jacobi_batched(int prec, int R, int G, int with_v, const JacobiJob* jobs_dev, const int* task_job,
                                 const int* task_slice, int ntasks, int* queue, int max_sweeps, Ctrl* ctrl,
                                 int lds_bytes, hipStream_t s);
// Row geometry of a tall m x p slice: G lanes per column pair (16 or 32), R
// rows per lane (4, 8, 12 or 16, R G >= m), ldv the padded V column length.
// jacobi_geometry picks the default G; jacobi_geometry_g returns -1 when G
// cannot hold m rows.
void jacobi_geometry(int m, int p, int* G, int* R, int* ldv);
int jacobi_geometry_g(int m, int p, int G, int* R, int* ldv);
int jacobi_resident_lds_bytes(int prec, int m, int p, int G, int with_v);
int jacobi_team_lds_bytes(int prec, int m, int p, int G, int b, int with_v);
int jacobi_team_max_resident(int prec, int lds_bytes, int threads, int with_v, int R, int G, int K);

}  // namespace tsvd
