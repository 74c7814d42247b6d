// Batched one-sided (Hestenes) Jacobi SVD of the transformed frontal slices.
//
// The method takes the SVD of every frontal slice of Zbar = dct(Z,[],3)
// (Theorem 4; Algorithm 1, per-slice SVD).  Each slice is handled in "tall"
// form T (m x p, m >= p): the slice itself, or its transpose when n1 < n2.
// Columns of T are rotated in pairs until every pair is orthogonal to
// tol = m * u (u = unit roundoff of the sweep arithmetic):
//     alpha = |x|^2, beta = |y|^2, gamma = x.y        (FP64 sums)
//     zeta = (beta - alpha) / (2 gamma),  t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2))
//     c = 1 / sqrt(1 + t^2),  s = c t,  x' = c x - s y,  y' = s x + c y.
// On exit A holds T V (columns = sigma_j u_j); V is accumulated only when asked.
//
// Two kernels share the pair routine:
//  * resident: one workgroup per slice, the whole slice (and V) in LDS, parallel
//    round-robin ordering over all columns (p/2 disjoint pairs per round, one
//    wavefront per pair, 64-lane shuffle reductions).
//  * team: slices too large for LDS.  Columns are cut into nb blocks of b; a
//    round-robin tournament over blocks gives nb/2 disjoint block pairs per
//    step.  W workgroups of a team each hold one block pair in LDS per step,
//    orthogonalize it (intra-block pairs on the first step of a sweep, then all
//    b*b cross pairs), write it back, and meet at a team barrier.  The grid is
//    launched cooperatively, so every workgroup of a team is resident; the
//    barrier's wait is bounded and reports a timeout instead of hanging.
#include "internal.h"

namespace tsvd {

template <typename T> struct Unit;
template <> struct Unit<double> { static constexpr double v = 1.1102230246251565e-16; };  // 2^-53
template <> struct Unit<float> { static constexpr double v = 5.9604644775390625e-08; };    // 2^-24

__device__ __forceinline__ double wave_sum(double v) {
    // Butterfly: every lane ends with the same bits (the adds are symmetric).
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Circle-method round robin on n (even) players: round s (0..n-2), pair q
// (0..n/2-1) -> players (i < j).  Every pair meets exactly once in n-1 rounds.
__device__ __forceinline__ void rr_pair(int s, int q, int n, int& i, int& j) {
    int a, b;
    if (q == 0) {
        a = n - 1;
        b = s;
    } else {
        a = (s + q) % (n - 1);
        b = (s - q + n - 1) % (n - 1);
    }
    i = a < b ? a : b;
    j = a < b ? b : a;
}

// Orthogonalize columns x, y (LDS, EPL*64 rows, zero padded) and rotate the V
// columns vx, vy (vrows rows, 0 = none).  f64 selects FP64 dots and rotation
// for float data (the refinement sweep).  Returns 1 if a rotation was applied.
template <typename T, int EPL>
__device__ __forceinline__ int jpair(T* __restrict__ x, T* __restrict__ y, T* __restrict__ vx,
                                     T* __restrict__ vy, int vrows, int lane, double tol, bool f64) {
    T xr[EPL], yr[EPL];
#pragma unroll
    for (int q = 0; q < EPL; ++q) {
        xr[q] = x[lane + kWave * q];
        yr[q] = y[lane + kWave * q];
    }
    double a, b, g;
    if (sizeof(T) == 8 || f64) {
        double pa = 0.0, pb = 0.0, pg = 0.0;
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
            double xd = (double)xr[q], yd = (double)yr[q];
            pa = fma(xd, xd, pa);
            pb = fma(yd, yd, pb);
            pg = fma(xd, yd, pg);
        }
        a = pa; b = pb; g = pg;
    } else {
        T pa = 0, pb = 0, pg = 0;
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
            pa = fmaf(xr[q], xr[q], pa);
            pb = fmaf(yr[q], yr[q], pb);
            pg = fmaf(xr[q], yr[q], pg);
        }
        a = (double)pa; b = (double)pb; g = (double)pg;
    }
    a = wave_sum(a);
    b = wave_sum(b);
    g = wave_sum(g);
    if (g == 0.0 || fabs(g) <= tol * sqrt(a) * sqrt(b)) return 0;
    const double zeta = (b - a) / (2.0 * g);
    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
    const double c = 1.0 / sqrt(1.0 + t * t);
    const double s = c * t;
    if (sizeof(T) == 8 || f64) {
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
            double xd = (double)xr[q], yd = (double)yr[q];
            x[lane + kWave * q] = (T)(c * xd - s * yd);
            y[lane + kWave * q] = (T)(s * xd + c * yd);
        }
        for (int r = lane; r < vrows; r += kWave) {
            double xd = (double)vx[r], yd = (double)vy[r];
            vx[r] = (T)(c * xd - s * yd);
            vy[r] = (T)(s * xd + c * yd);
        }
    } else {
        const T cc = (T)c, ss = (T)s;
#pragma unroll
        for (int q = 0; q < EPL; ++q) {
            x[lane + kWave * q] = cc * xr[q] - ss * yr[q];
            y[lane + kWave * q] = ss * xr[q] + cc * yr[q];
        }
        for (int r = lane; r < vrows; r += kWave) {
            T xd = vx[r], yd = vy[r];
            vx[r] = cc * xd - ss * yd;
            vy[r] = ss * xd + cc * yd;
        }
    }
    return 1;
}

// Element (r, c) of slice k's tall matrix in the source tensor.
template <typename T>
__device__ __forceinline__ T src_at(const JacobiJob& J, int k, int r, int c) {
    return ((const T*)J.src)[(int64_t)k * J.src_ss + (int64_t)r * J.src_rs + (int64_t)c * J.src_cs];
}

__device__ __forceinline__ int block_sum_int(int v, int* s_scratch) {
    // v is per-wave (uniform within a wave); lane 0 of each wave contributes.
    if (threadIdx.x == 0) *s_scratch = 0;
    __syncthreads();
    if ((threadIdx.x & (kWave - 1)) == 0 && v) atomicAdd(s_scratch, v);
    __syncthreads();
    int tot = *s_scratch;
    __syncthreads();
    return tot;
}

// ---------------------------------------------------------------------------
// Resident kernel: one workgroup per (job, slice) task, whole slice in LDS.
// LDS: pp columns of ldl = 64*EPL rows of A, then (with V) pp columns of p rows.
// ---------------------------------------------------------------------------
template <typename T, int EPL, bool WV>
__device__ void resident_task(const JacobiJob& J, int k, int max_sweeps, Ctrl* ctrl, T* lds, int* s_scratch) {
    const int m = J.m, p = J.p;
    const int ldl = kWave * EPL;
    const int pp = p + (p & 1);
    T* As = lds;
    T* Vs = lds + (int64_t)pp * ldl;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int wave = tid / kWave, lane = tid % kWave, NW = nth / kWave;

    if (J.src_rs == 1) {
        for (int e = tid; e < pp * ldl; e += nth) {
            int c = e / ldl, r = e - c * ldl;
            As[e] = (c < p && r < m) ? src_at<T>(J, k, r, c) : (T)0;
        }
    } else {  // transposed source: walk columns fastest for contiguous reads
        for (int e = tid; e < pp * ldl; e += nth) {
            int r = e / pp, c = e - r * pp;
            As[c * ldl + r] = (c < p && r < m) ? src_at<T>(J, k, r, c) : (T)0;
        }
    }
    if (WV)
        for (int e = tid; e < pp * p; e += nth) {
            int c = e / p, r = e - c * p;
            Vs[e] = (r == c) ? (T)1 : (T)0;
        }
    __syncthreads();

    const double tol = (double)m * Unit<T>::v;
    int sweeps = -1, executed = 0;
    bool refine = J.refine64 != 0;
    for (int sw = 0; sw < max_sweeps + (refine ? 1 : 0); ++sw) {
        const bool f64 = refine && sw == max_sweeps;  // only reached via the refinement path below
        int rot = 0;
        ++executed;
        for (int s = 0; s < pp - 1; ++s) {
            for (int q = wave; q < pp / 2; q += NW) {
                int i, j;
                rr_pair(s, q, pp, i, j);
                if (j < p)
                    rot += jpair<T, EPL>(As + i * ldl, As + j * ldl, WV ? Vs + i * p : nullptr,
                                         WV ? Vs + j * p : nullptr, WV ? p : 0, lane,
                                         f64 ? (double)m * Unit<double>::v : tol, f64);
            }
            __syncthreads();
        }
        int tot = block_sum_int(rot, s_scratch);
        if (f64) break;
        if (tot == 0) {
            sweeps = sw + 1;
            if (!refine) break;
            // one refinement sweep in FP64 arithmetic, then stop
            sw = max_sweeps - 1;
        }
    }
    // write back A (and V)
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    for (int e = tid; e < p * m; e += nth) {
        int c = e / m, r = e - c * m;
        Ag[e] = As[c * ldl + r];
    }
    if (WV) {
        T* Vg = (T*)J.V + (int64_t)k * p * p;
        for (int e = tid; e < p * p; e += nth) Vg[e] = Vs[e];
    }
    if (tid == 0) {
        J.sweeps[k] = sweeps;
        if (sweeps < 0) atomicOr(&ctrl->status, kStNoConv);
        else atomicMax(&ctrl->max_sweeps, sweeps);
        atomicAdd(&ctrl->slice_sweeps, (unsigned long long)executed);
    }
}

template <typename T, bool WV>
__global__ __launch_bounds__(1024) void k_jacobi_resident(const JacobiJob* __restrict__ jobs,
                                                          const int* __restrict__ task_job,
                                                          const int* __restrict__ task_slice, int ntasks,
                                                          int max_sweeps, Ctrl* ctrl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_scratch;
    T* lds = (T*)smem_raw;
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        const JacobiJob& J = jobs[task_job[t]];
        const int k = task_slice[t];
        switch (J.epl) {
            case 1: resident_task<T, 1, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
            case 2: resident_task<T, 2, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
            case 3: resident_task<T, 3, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
            case 4: resident_task<T, 4, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
            case 5: resident_task<T, 5, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
            case 6: resident_task<T, 6, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
            case 7: resident_task<T, 7, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
            default: resident_task<T, 8, WV>(J, k, max_sweeps, ctrl, lds, &s_scratch); break;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Team kernel.
// ---------------------------------------------------------------------------
struct TeamState {
    int* bar;       // this team's barrier counter
    int passed;     // barriers passed so far by this workgroup
    int W;
    int spin_limit;
    Ctrl* ctrl;
};

// Returns false when the wait gave up (the caller then abandons the launch).
__device__ bool team_barrier(TeamState& ts, int* s_flag) {
    __threadfence();  // release this thread's global writes at device scope
    __syncthreads();
    ts.passed += 1;
    if (threadIdx.x == 0) {
        *s_flag = 0;
        if (ts.W > 1) {
            __hip_atomic_fetch_add(ts.bar, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const int target = ts.passed * ts.W;
            int it = 0;
            while (__hip_atomic_load(ts.bar, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (++it > ts.spin_limit) {
                    atomicOr(&ts.ctrl->status, kStTimeout);
                    *s_flag = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
    }
    __syncthreads();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    const bool ok = (*s_flag == 0);
    __syncthreads();
    return ok;
}

template <typename T, int EPL, bool WV>
__device__ __forceinline__ void team_load_block(const JacobiJob& J, int k, int blk, bool first, T* As, T* Vs) {
    const int m = J.m, p = J.p, b = J.b, ldl = kWave * EPL;
    const int tid = threadIdx.x, nth = blockDim.x;
    const T* Ag = (const T*)J.A + (int64_t)k * m * p;
    if (first && J.src_rs != 1) {
        for (int e = tid; e < b * ldl; e += nth) {
            int r = e / b, cl = e - r * b, c = blk * b + cl;
            As[cl * ldl + r] = (c < p && r < m) ? src_at<T>(J, k, r, c) : (T)0;
        }
    } else {
        for (int e = tid; e < b * ldl; e += nth) {
            int cl = e / ldl, r = e - cl * ldl, c = blk * b + cl;
            T v = (T)0;
            if (c < p && r < m) v = first ? src_at<T>(J, k, r, c) : Ag[(int64_t)c * m + r];
            As[e] = v;
        }
    }
    if (WV) {
        const T* Vg = (const T*)J.V + (int64_t)k * p * p;
        for (int e = tid; e < b * p; e += nth) {
            int cl = e / p, r = e - cl * p, c = blk * b + cl;
            T v = (T)0;
            if (c < p) v = first ? (T)(r == c ? 1 : 0) : Vg[(int64_t)c * p + r];
            Vs[e] = v;
        }
    }
}

template <typename T, int EPL, bool WV>
__device__ __forceinline__ void team_store_block(const JacobiJob& J, int k, int blk, const T* As, const T* Vs) {
    const int m = J.m, p = J.p, b = J.b, ldl = kWave * EPL;
    const int tid = threadIdx.x, nth = blockDim.x;
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    for (int e = tid; e < b * m; e += nth) {
        int cl = e / m, r = e - cl * m, c = blk * b + cl;
        if (c < p) Ag[(int64_t)c * m + r] = As[cl * ldl + r];
    }
    if (WV) {
        T* Vg = (T*)J.V + (int64_t)k * p * p;
        for (int e = tid; e < b * p; e += nth) {
            int cl = e / p, r = e - cl * p, c = blk * b + cl;
            if (c < p) Vg[(int64_t)c * p + r] = Vs[e];
        }
    }
}

// Returns false if a barrier timed out.
template <typename T, int EPL, bool WV>
__device__ bool team_task(const JacobiJob& J, int k, int rank, TeamState& ts, int max_sweeps, T* lds,
                          int* s_scratch, int* s_flag) {
    const int m = J.m, p = J.p, b = J.b, nb = J.nb, ldl = kWave * EPL;
    const int tid = threadIdx.x;
    const int wave = tid / kWave, lane = tid % kWave, NW = blockDim.x / kWave;
    T* As = lds;                            // 2b columns x ldl
    T* Vs = lds + (int64_t)2 * b * ldl;     // 2b columns x p
    const double tol = (double)m * Unit<T>::v;
    const bool refine = J.refine64 != 0;
    int sweeps = -1, executed = 0;
    int* rot_g = J.rot + (int64_t)k * kMaxSweeps;
    for (int sw = 0; sw < max_sweeps + (refine ? 1 : 0); ++sw) {
        const bool f64 = refine && sw == max_sweeps;
        const double tl = f64 ? (double)m * Unit<double>::v : tol;
        int rot = 0;
        ++executed;
        for (int s = 0; s < nb - 1; ++s) {
            for (int q = rank; q < nb / 2; q += ts.W) {
                int BI, BJ;
                rr_pair(s, q, nb, BI, BJ);
                const bool first = (sw == 0 && s == 0);
                team_load_block<T, EPL, WV>(J, k, BI, first, As, Vs);
                team_load_block<T, EPL, WV>(J, k, BJ, first, As + b * ldl, Vs + b * p);
                __syncthreads();
                if (s == 0) {
                    // intra-block pairs of both blocks: b-1 rounds of b pairs
                    for (int r = 0; r < b - 1; ++r) {
                        for (int q2 = wave; q2 < b; q2 += NW) {
                            const int half = q2 < b / 2 ? 0 : 1;
                            int i, j;
                            rr_pair(r, q2 - half * (b / 2), b, i, j);
                            const int blk = half ? BJ : BI;
                            if (blk * b + j < p) {
                                const int off = half * b;
                                rot += jpair<T, EPL>(As + (off + i) * ldl, As + (off + j) * ldl,
                                                     WV ? Vs + (off + i) * p : nullptr,
                                                     WV ? Vs + (off + j) * p : nullptr, WV ? p : 0, lane, tl, f64);
                            }
                        }
                        __syncthreads();
                    }
                }
                // cross pairs: b rounds of b disjoint pairs (I[i], J[(i + r) % b])
                for (int r = 0; r < b; ++r) {
                    for (int i = wave; i < b; i += NW) {
                        const int j = (i + r) % b;
                        if (BI * b + i < p && BJ * b + j < p)
                            rot += jpair<T, EPL>(As + i * ldl, As + (b + j) * ldl, WV ? Vs + i * p : nullptr,
                                                 WV ? Vs + (b + j) * p : nullptr, WV ? p : 0, lane, tl, f64);
                    }
                    __syncthreads();
                }
                team_store_block<T, EPL, WV>(J, k, BI, As, Vs);
                team_store_block<T, EPL, WV>(J, k, BJ, As + b * ldl, Vs + b * p);
                __syncthreads();
            }
            if (s == nb - 2) {
                int tot = block_sum_int(rot, s_scratch);
                if (tid == 0 && tot) atomicAdd(rot_g + sw, tot);
            }
            if (!team_barrier(ts, s_flag)) return false;
        }
        if (f64) break;
        const int total = __hip_atomic_load(rot_g + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (total == 0) {
            sweeps = sw + 1;
            if (!refine) break;
            sw = max_sweeps - 1;
        }
    }
    if (tid == 0 && rank == 0) {
        J.sweeps[k] = sweeps;
        if (sweeps < 0) atomicOr(&ts.ctrl->status, kStNoConv);
        else atomicMax(&ts.ctrl->max_sweeps, sweeps);
        atomicAdd(&ts.ctrl->slice_sweeps, (unsigned long long)executed);
    }
    return true;
}

template <typename T, bool WV>
__global__ __launch_bounds__(1024) void k_jacobi_team(const JacobiJob* __restrict__ jobs,
                                                      const int* __restrict__ task_job,
                                                      const int* __restrict__ task_slice, int ntasks,
                                                      TeamSched sched, int max_sweeps, Ctrl* ctrl,
                                                      int spin_limit) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_scratch, s_flag;
    T* lds = (T*)smem_raw;
    const int W = sched.W;
    const int team = blockIdx.x / W, rank = blockIdx.x % W;
    if (team >= sched.nteams) return;
    TeamState ts{sched.bar + team, 0, W, spin_limit, ctrl};
    for (int t = team; t < ntasks; t += sched.nteams) {
        const JacobiJob& J = jobs[task_job[t]];
        const int k = task_slice[t];
        bool ok;
        switch (J.epl) {
            case 1: ok = team_task<T, 1, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
            case 2: ok = team_task<T, 2, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
            case 3: ok = team_task<T, 3, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
            case 4: ok = team_task<T, 4, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
            case 5: ok = team_task<T, 5, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
            case 6: ok = team_task<T, 6, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
            case 7: ok = team_task<T, 7, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
            default: ok = team_task<T, 8, WV>(J, k, rank, ts, max_sweeps, lds, &s_scratch, &s_flag); break;
        }
        if (!ok) return;
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int elem_size(int prec) { return prec == 0 ? 8 : 4; }

int jacobi_resident_lds_bytes(int prec, int m, int p, int with_v) {
    const int epl = (m + kWave - 1) / kWave;
    const int pp = p + (p & 1);
    int64_t elems = (int64_t)pp * epl * kWave + (with_v ? (int64_t)pp * p : 0);
    return (int)(elems * elem_size(prec));
}

int jacobi_team_lds_bytes(int prec, int m, int p, int b, int with_v) {
    const int epl = (m + kWave - 1) / kWave;
    int64_t elems = (int64_t)2 * b * epl * kWave + (with_v ? (int64_t)2 * b * p : 0);
    return (int)(elems * elem_size(prec));
}

template <typename T, bool WV>
static hipError_t set_lds_attr_team(int lds) {
    return hipFuncSetAttribute((const void*)k_jacobi_team<T, WV>, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}
template <typename T, bool WV>
static hipError_t set_lds_attr_res(int lds) {
    return hipFuncSetAttribute((const void*)k_jacobi_resident<T, WV>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               lds);
}

hipError_t launch_jacobi_resident(int prec, const JacobiJob* jobs_dev, int njobs, const int* task_job,
                                  const int* task_slice, int ntasks, int max_sweeps, Ctrl* ctrl, int lds_bytes,
                                  int threads, int with_v, hipStream_t s) {
    (void)njobs;
    if (ntasks <= 0) return hipSuccess;
    dim3 grid(ntasks), block(threads);
    hipError_t e;
    if (prec == 0) {
        if (with_v) {
            if ((e = set_lds_attr_res<double, true>(lds_bytes)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_jacobi_resident<double, true>), grid, block, lds_bytes, s, jobs_dev, task_job,
                               task_slice, ntasks, max_sweeps, ctrl);
        } else {
            if ((e = set_lds_attr_res<double, false>(lds_bytes)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_jacobi_resident<double, false>), grid, block, lds_bytes, s, jobs_dev, task_job,
                               task_slice, ntasks, max_sweeps, ctrl);
        }
    } else {
        if (with_v) {
            if ((e = set_lds_attr_res<float, true>(lds_bytes)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_jacobi_resident<float, true>), grid, block, lds_bytes, s, jobs_dev, task_job,
                               task_slice, ntasks, max_sweeps, ctrl);
        } else {
            if ((e = set_lds_attr_res<float, false>(lds_bytes)) != hipSuccess) return e;
            hipLaunchKernelGGL((k_jacobi_resident<float, false>), grid, block, lds_bytes, s, jobs_dev, task_job,
                               task_slice, ntasks, max_sweeps, ctrl);
        }
    }
    return hipGetLastError();
}

template <typename T, bool WV>
static hipError_t coop_team(const JacobiJob* jobs_dev, const int* task_job, const int* task_slice, int ntasks,
                            TeamSched ts, int max_sweeps, Ctrl* ctrl, int lds, int threads, int spin_limit,
                            hipStream_t s) {
    hipError_t e = set_lds_attr_team<T, WV>(lds);
    if (e != hipSuccess) return e;
    void* args[] = {(void*)&jobs_dev, (void*)&task_job, (void*)&task_slice, (void*)&ntasks,
                    (void*)&ts,       (void*)&max_sweeps, (void*)&ctrl,     (void*)&spin_limit};
    dim3 grid(ts.nteams * ts.W), block(threads);
    return hipLaunchCooperativeKernel((const void*)k_jacobi_team<T, WV>, grid, block, args, (unsigned)lds, s);
}

hipError_t launch_jacobi_team(int prec, const JacobiJob* jobs_dev, int njobs, const int* task_job,
                              const int* task_slice, int ntasks, const TeamSched& ts, int max_sweeps, Ctrl* ctrl,
                              int lds_bytes, int threads, int with_v, int spin_limit, hipStream_t s) {
    (void)njobs;
    if (ntasks <= 0) return hipSuccess;
    if (prec == 0)
        return with_v ? coop_team<double, true>(jobs_dev, task_job, task_slice, ntasks, ts, max_sweeps, ctrl,
                                                lds_bytes, threads, spin_limit, s)
                      : coop_team<double, false>(jobs_dev, task_job, task_slice, ntasks, ts, max_sweeps, ctrl,
                                                 lds_bytes, threads, spin_limit, s);
    return with_v ? coop_team<float, true>(jobs_dev, task_job, task_slice, ntasks, ts, max_sweeps, ctrl, lds_bytes,
                                           threads, spin_limit, s)
                  : coop_team<float, false>(jobs_dev, task_job, task_slice, ntasks, ts, max_sweeps, ctrl, lds_bytes,
                                            threads, spin_limit, s);
}

int jacobi_team_max_resident(int prec, int lds_bytes, int threads, int with_v) {
    int nb = 0;
    hipError_t e;
    const void* f = prec == 0 ? (with_v ? (const void*)k_jacobi_team<double, true> : (const void*)k_jacobi_team<double, false>)
                              : (with_v ? (const void*)k_jacobi_team<float, true> : (const void*)k_jacobi_team<float, false>);
    e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // do not leave a sticky error for the caller's runtime
        return 0;
    }
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, threads, lds_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return nb * cus;
}

}  // namespace tsvd
