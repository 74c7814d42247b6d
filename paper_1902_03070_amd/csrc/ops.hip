// Tube transforms, batched slice GEMMs and the thresholding step.
#include <algorithm>
#include "internal.h"

namespace tsvd {

// ---------------------------------------------------------------------------
// Tube transform: out[r + N k'] = sum_k M[k'][k] in[r + N k]   (r < N = n1 n2)
// With M = C this is Zbar = dct(Z,[],3) (Section 3); with M = C^T it is the
// inverse.  Workgroup: 64 consecutive tubes x 4 wavefronts.  The 64 x n3 input
// tile is staged in LDS; each wavefront produces KB outputs per pass for its
// 64 tubes, reading the transform row from scalar memory (wave-uniform).
// Optional prologue (completion): in = X - Mlt/beta.
// Optional epilogue (completion, Algorithm 1 X- and M-updates):
//   Xn = mask ? B : y + Mlt/beta;  Mlt += beta (y - Xn);  X = Xn
// with FP64 partial sums of ||Xn - X||^2 and ||X||^2.
// ---------------------------------------------------------------------------
constexpr int kTubeKB = 8;

__device__ __forceinline__ double beta_of(const TubeArgs& a) {
    return a.beta_sched ? a.beta_sched[a.ctrl->iter] : a.beta_val;
}

template <typename T>
__global__ __launch_bounds__(256) void k_tube(TubeArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double s_red[2][4];
    T* tile = (T*)smem_raw;  // n3 x 64
    const int n3 = a.n3;
    const int64_t N = a.N;
    const int tl = threadIdx.x % kTubeTile;
    const int grp = __builtin_amdgcn_readfirstlane(threadIdx.x / kTubeTile);  // one wavefront per group
    const int64_t r = (int64_t)blockIdx.x * kTubeTile + tl;
    const bool live = r < N;
    const T* Mx = (const T*)a.M;

    double beta = 1.0;
    if (a.pX || a.eX) beta = beta_of(a);

    int bad = 0;
    for (int k = grp; k < n3; k += 4) {
        T v = (T)0;
        if (live) {
            const int64_t e = r + N * k;
            if (a.pX) {
                v = (T)((double)((const T*)a.pX)[e] - (double)((const T*)a.pM)[e] / beta);
            } else {
                v = ((const T*)a.in)[e];
            }
            if (a.check_finite && !isfinite((double)v)) bad = 1;
        }
        tile[k * kTubeTile + tl] = v;
    }
    if (a.check_finite && bad) atomicOr(&a.ctrl->status, kStNonFinite);
    __syncthreads();

    double dn = 0.0, xn = 0.0;
    for (int kb = grp * kTubeKB; kb < n3; kb += 4 * kTubeKB) {
        T acc[kTubeKB];
#pragma unroll
        for (int u = 0; u < kTubeKB; ++u) acc[u] = (T)0;
        for (int t = 0; t < n3; ++t) {
            const T x = tile[t * kTubeTile + tl];
#pragma unroll
            for (int u = 0; u < kTubeKB; ++u) {
                const int row = min(kb + u, n3 - 1);
                acc[u] = fma(Mx[row * n3 + t], x, acc[u]);
            }
        }
        if (live) {
#pragma unroll
            for (int u = 0; u < kTubeKB; ++u) {
                const int ko = kb + u;
                if (ko >= n3) break;
                const int64_t e = r + N * ko;
                const T y = acc[u];
                if (a.out) ((T*)a.out)[e] = y;
                if (a.eX) {
                    T* X = (T*)a.eX;
                    T* Ml = (T*)a.eM;
                    const T xold = X[e];
                    const T mold = Ml[e];
                    T xnew;
                    if (a.emask[e]) xnew = ((const T*)a.eB)[e];
                    else xnew = (T)((double)y + (double)mold / beta);
                    Ml[e] = (T)((double)mold + beta * ((double)y - (double)xnew));
                    X[e] = xnew;
                    const double d = (double)xnew - (double)xold;
                    dn += d * d;
                    xn += (double)xold * (double)xold;
                }
            }
        }
    }
    if (a.eX && a.norms) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dn += __shfl_xor(dn, o, kWave);
            xn += __shfl_xor(xn, o, kWave);
        }
        if (tl == 0) {
            s_red[0][grp] = dn;
            s_red[1][grp] = xn;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double* slot = a.norms + 2 * (blockIdx.x % kNormSlots);
            atomicAdd(slot, s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3]);
            atomicAdd(slot + 1, s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3]);
        }
    }
}

hipError_t launch_tube_transform(int prec, const TubeArgs& a, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.N + kTubeTile - 1) / kTubeTile)), block(256);
    const int lds = dense_tube_lds(prec, a.n3);
    if (lds > kLdsBudget) return hipErrorInvalidValue;
    if (prec == 0) hipLaunchKernelGGL(k_tube<double>, grid, block, lds, s, a);
    else hipLaunchKernelGGL(k_tube<float>, grid, block, lds, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched strided GEMM  C_b = (A_b B_b) diag(cscale_b), K_b from Kdev or K,
// on the matrix cores (v_mfma_f32_16x16x4f32 / v_mfma_f64_16x16x4f64).
// A workgroup of 256 threads computes a 64 x 64 tile of C; wavefront w takes
// the 32 x 32 quarter (w & 1, w >> 1) as 2 x 2 blocks of 16 x 16.  K goes
// through LDS in chunks of 32, and the next chunk's global loads are issued
// before the current chunk's products.  Each block is formed as
// C^T = B^T A^T, so the 16 lanes of a result row run down a column of C
// (contiguous stores for column-major C).
//
// Lane layouts (gfx950): A 16xK operand, lane l holds row l%16 and K slice
// l/16; B Kx16 operand, lane l holds column l%16 and K slice l/16; result:
// FP64 element v of lane l is row l/16 + 4v, FP32 element v is row
// 4(l/16) + v, column l%16 in both.
// ---------------------------------------------------------------------------
typedef double gd4_t __attribute__((ext_vector_type(4)));
typedef float gf4_t __attribute__((ext_vector_type(4)));
template <typename T> struct GemmAcc;
template <> struct GemmAcc<double> { typedef gd4_t V; };
template <> struct GemmAcc<float> { typedef gf4_t V; };

constexpr int kGemmKT = 32;  // K chunk staged in LDS

template <typename T>
__device__ __forceinline__ typename GemmAcc<T>::V mfma16x16x4(T a, T b, typename GemmAcc<T>::V c) {
    if constexpr (sizeof(T) == 8) return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    else return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Element q (< 8) of thread tid in a 64 x 32 (A) or 32 x 64 (B) chunk: the
// index pairs run along the operand's unit-stride dimension for coalescing.
__device__ __forceinline__ void gemm_chunk_index(int e, bool along64, int& x64, int& x32) {
    if (along64) { x64 = e & 63; x32 = e >> 6; }
    else { x32 = e & 31; x64 = e >> 5; }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    constexpr int LD = 64 + (sizeof(T) == 4 ? 16 : 8);  // row pitch: 16-lane runs of adjacent rows fall in different banks
    __shared__ T As[kGemmKT][LD];  // As[k][i]
    __shared__ T Bs[kGemmKT][LD];  // Bs[k][j]
    typedef typename GemmAcc<T>::V Acc;
    const int b = blockIdx.z;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int K = g.Kdev ? g.Kdev[b] : g.K;
    const int Nb = g.Ndev ? g.Ndev[b] : g.Nn;
    if (j0 >= Nb) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    const int wi = (w & 1) * 32, wj = (w >> 1) * 32;
    const T* A = (const T*)g.A + (int64_t)b * g.a_bs;
    const T* B = (const T*)g.B + (int64_t)b * g.b_bs;
    const bool a_rowfast = g.a_rs == 1;
    const bool b_kfast = g.b_rs == 1;
    T ra[8], rb[8];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            int ii, tt, jj, tb;
            gemm_chunk_index(e, a_rowfast, ii, tt);
            gemm_chunk_index(e, !b_kfast, jj, tb);
            const int gi = i0 + ii, gt = t0 + tt, gj = j0 + jj, gtb = t0 + tb;
            ra[q] = (gi < g.M && gt < K) ? A[(int64_t)gi * g.a_rs + (int64_t)gt * g.a_cs] : (T)0;
            rb[q] = (gj < Nb && gtb < K) ? B[(int64_t)gtb * g.b_rs + (int64_t)gj * g.b_cs] : (T)0;
        }
    };
    Acc acc[2][2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int v = 0; v < 2; ++v)
#pragma unroll
            for (int e = 0; e < 4; ++e) acc[u][v][e] = (T)0;
    if (K > 0) fetch(0);
    for (int t0 = 0; t0 < K; t0 += kGemmKT) {
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int e = tid + 256 * q;
            int ii, tt, jj, tb;
            gemm_chunk_index(e, a_rowfast, ii, tt);
            gemm_chunk_index(e, !b_kfast, jj, tb);
            As[tt][ii] = ra[q];
            Bs[tb][jj] = rb[q];
        }
        __syncthreads();
        if (t0 + kGemmKT < K) fetch(t0 + kGemmKT);
#pragma unroll
        for (int ks = 0; ks < kGemmKT; ks += 4) {
            const int kk = ks + (lane >> 4);
            T af[2], bf[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) af[u] = As[kk][wi + 16 * u + (lane & 15)];
#pragma unroll
            for (int v = 0; v < 2; ++v) bf[v] = Bs[kk][wj + 16 * v + (lane & 15)];
#pragma unroll
            for (int u = 0; u < 2; ++u)
#pragma unroll
                for (int v = 0; v < 2; ++v) acc[u][v] = mfma16x16x4<T>(bf[v], af[u], acc[u][v]);
        }
        __syncthreads();
    }
    T* C = (T*)g.C + (int64_t)b * g.c_bs;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int i = i0 + wi + 16 * u + (lane & 15);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int jr = sizeof(T) == 8 ? (lane >> 4) + 4 * e : 4 * (lane >> 4) + e;
                const int j = j0 + wj + 16 * v + jr;
                if (i >= g.M || j >= Nb) continue;
                const T val = acc[u][v][e];
                C[(int64_t)i * g.c_rs + (int64_t)j * g.c_cs] =
                    g.cscale ? (T)((double)val * g.cscale[(int64_t)b * g.s_bs + j]) : val;
            }
        }
    }
}

hipError_t launch_gemm(int prec, const GemmArgs& g, hipStream_t s) {
    if (g.M <= 0 || g.Nn <= 0 || g.batch <= 0) return hipSuccess;
    dim3 grid((g.M + 63) / 64, (g.Nn + 63) / 64, g.batch), block(256);
    if (prec == 0) hipLaunchKernelGGL(k_gemm<double>, grid, block, 0, s, g);
    else hipLaunchKernelGGL(k_gemm<float>, grid, block, 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Thresholding (Theorem 5): per slice, sigma_c = ||A'(:,c)|| (FP64), keep the
// columns with sigma_c > tau in index order, copy them to F, and set
// w_q = (sigma_c - tau) / sigma_c^3 so that the rebuilt slice is
//   Ybar = F diag(w) F^T Zbar            (tall form)
// since A' = T V has columns a_c = sigma_c u_c and a_c^T T = sigma_c^2 v_c^T,
// so (sigma_c - tau) u_c v_c^T = w_c a_c a_c^T T.
// One workgroup (256 threads) per slice.
// ---------------------------------------------------------------------------
// Three launches, each spread over (column groups, slices):
//   norms:  sigma_c = |A'(:,c)| for every column (one wavefront per column);
//   select: per slice, keep = sigma > tau, positions of the kept columns in
//           order (a wavefront ballot), rank, w_q = (sigma - tau) / sigma^3;
//   gather: copy each kept column of A' to its position in F.
template <typename T>
__global__ __launch_bounds__(256) void k_svt_norms(SvtPrepArgs a) {
    const int k = blockIdx.y, lane = threadIdx.x % kWave;
    const int c = blockIdx.x * 4 + threadIdx.x / kWave;
    if (c >= a.p) return;
    const T* col = (const T*)a.A + (int64_t)k * a.a_ss + (int64_t)c * a.m;
    double acc = 0.0;
    for (int r = lane; r < a.m; r += kWave) {
        const double v = (double)col[r];
        acc = fma(v, v, acc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (lane == 0) a.sig[(int64_t)k * a.sig_ss + c] = sqrt(acc);
}

__global__ __launch_bounds__(64) void k_svt_select(SvtPrepArgs a) {
    const int k = blockIdx.x, lane = threadIdx.x;
    const double tau = a.tau_sched ? a.tau_sched[a.ctrl->iter] : a.tau_val;
    const double* sig = a.sig + (int64_t)k * a.sig_ss;
    int* pos = a.pos + (int64_t)k * a.p;
    int base = 0;
    for (int c0 = 0; c0 < a.p; c0 += kWave) {
        const int c = c0 + lane;
        const double sg = c < a.p ? sig[c] : 0.0;
        const bool keep = c < a.p && sg > tau;
        const unsigned long long mask = __ballot(keep);
        const int q = base + __popcll(mask & ((1ull << lane) - 1ull));
        if (c < a.p) pos[c] = keep ? q : -1;
        if (keep) a.w[(int64_t)k * a.w_ss + q] = ((sg - tau) / sg) / sg / sg;
        base += __popcll(mask);
    }
    if (lane == 0) a.ranks[k] = base;
}

template <typename T>
__global__ __launch_bounds__(256) void k_svt_gather(SvtPrepArgs a) {
    const int k = blockIdx.y, lane = threadIdx.x % kWave;
    const int c = blockIdx.x * 4 + threadIdx.x / kWave;
    if (c >= a.p) return;
    const int q = a.pos[(int64_t)k * a.p + c];
    if (q < 0) return;
    const T* src = (const T*)a.A + (int64_t)k * a.a_ss + (int64_t)c * a.m;
    T* dst = (T*)a.F + (int64_t)k * a.f_ss + (int64_t)q * a.m;
    for (int r = lane; r < a.m; r += kWave) dst[r] = src[r];
}

hipError_t launch_svt_prep(int prec, const SvtPrepArgs& a, hipStream_t s) {
    if (a.n3 <= 0 || a.p <= 0) return hipSuccess;
    const dim3 grid((a.p + 3) / 4, a.n3);
    if (prec == 0) hipLaunchKernelGGL(k_svt_norms<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_svt_norms<float>, grid, dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_svt_select, dim3(a.n3), dim3(kWave), 0, s, a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (prec == 0) hipLaunchKernelGGL(k_svt_gather<double>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_svt_gather<float>, grid, dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// t-SVD finish: order each slice's singular values descending (ties by column
// index), U(:,pos) = A'(:,c)/sigma_c, V(:,pos) = V_jacobi(:,c), and flip each
// pair so the largest-magnitude entry of U(:,pos) (first on ties) is positive.
// One workgroup per slice.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_tsvd_finish(TsvdFinishArgs a) {
    __shared__ double s_sig[kMaxRows];
    __shared__ int s_pos[kMaxRows];
    const int k = blockIdx.x, m = a.m, p = a.p;
    const int tid = threadIdx.x, lane = tid % kWave, wave = tid / kWave;
    for (int c = tid; c < p; c += blockDim.x) s_sig[c] = a.sig[(int64_t)k * a.sig_ss + c];
    __syncthreads();
    for (int c = tid; c < p; c += blockDim.x) {
        const double sc = s_sig[c];
        int pos = 0;
        for (int d = 0; d < p; ++d) {
            const double sd = s_sig[d];
            pos += (sd > sc || (sd == sc && d < c)) ? 1 : 0;
        }
        s_pos[c] = pos;
        ((T*)a.S)[(int64_t)k * a.s_ss + pos] = (T)sc;
    }
    __syncthreads();
    const T* A = (const T*)a.A + (int64_t)k * a.a_ss;
    const T* Vj = (const T*)a.Vj + (int64_t)k * a.v_ss;
    T* U = (T*)a.Ut + (int64_t)k * a.ut_ss;
    T* V = (T*)a.Vt + (int64_t)k * a.vt_ss;
    for (int c = wave; c < p; c += 4) {
        const double sc = s_sig[c];
        const double inv = sc > 0.0 ? 1.0 / sc : 0.0;
        // the slice's left singular vector is A(:,c) (tall) or V(:,c) (wide):
        // argmax of its magnitudes, first index on ties, decides the sign
        const T* L = a.sign_from_v ? Vj + (int64_t)c * p : A + (int64_t)c * m;
        const int nl = a.sign_from_v ? p : m;
        double best = -1.0;
        int bi = 0x7fffffff;
        for (int r = lane; r < nl; r += kWave) {
            const double v = fabs((double)L[r]);
            if (v > best) { best = v; bi = r; }
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(best, o, kWave);
            const int oi = __shfl_xor(bi, o, kWave);
            if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
        }
        const double sgn = (bi < nl && (double)L[bi] < 0.0) ? -1.0 : 1.0;
        const int pos = s_pos[c];
        for (int r = lane; r < m; r += kWave) U[(int64_t)pos * m + r] = (T)(sgn * inv * (double)A[(int64_t)c * m + r]);
        for (int r = lane; r < p; r += kWave) V[(int64_t)pos * p + r] = (T)(sgn * (double)Vj[(int64_t)c * p + r]);
    }
}

// ---------------------------------------------------------------------------
// Completion of the t-SVD's tall-side vectors (Theorem 4's full factors, and
// the columns of zero singular values).  One workgroup per slice, FP64
// arithmetic.  Column c is filled with the standard basis vector e_i whose
// part outside the span of the columns before it is largest (1 - sum_q
// Q[i][q]^2, first i on ties), projected out twice (Gram-Schmidt, each pass
// d = Q^T u, u -= Q d) and normalized.  Zero singular values (sorted last
// among the first p columns) get the sign convention of their pair (u_j,
// v_j); the full factor's columns p..m-1 get their largest entry positive.
// ---------------------------------------------------------------------------
__device__ double block_sum_d(double v, double* red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

// Load of a column this workgroup itself stored earlier in the kernel: an
// agent-scope relaxed load, which skips the CU's L1 (a line of it may still
// hold what was there before the store) and reads the L2.
template <typename T>
__device__ __forceinline__ double ld_fresh(const T* p) {
    return (double)__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Index of the largest v_r (largest |v_r| when absv; first on ties) over r < n,
// in every thread.
__device__ int block_argmax(const double* v, int n, bool absv, double* redv, int* redi) {
    const int tid = threadIdx.x;
    double best = -1e300;
    int bi = 0x7fffffff;
    for (int r = tid; r < n; r += blockDim.x) {
        const double x = absv ? fabs(v[r]) : v[r];
        if (x > best) { best = x; bi = r; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, kWave);
        const int oi = __shfl_xor(bi, o, kWave);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    __syncthreads();
    if ((tid & 63) == 0) { redv[tid >> 6] = best; redi[tid >> 6] = bi; }
    __syncthreads();
    best = redv[0];
    bi = redi[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
        if (redv[w] > best || (redv[w] == best && redi[w] < bi)) { best = redv[w]; bi = redi[w]; }
    return bi;
}

// Unit vector (in u) orthogonal to columns [0, nq) of Q (m rows, ld m), from
// the standard basis vector of largest residual.
template <typename T>
__device__ void complement_vector(const T* Q, int m, int nq, double* u, double* d, double* red, int* redi) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int r = tid; r < m; r += nt) {
        double acc = 0.0;
        for (int q = 0; q < nq; ++q) {
            const double x = ld_fresh(Q + (int64_t)q * m + r);
            acc = fma(x, x, acc);
        }
        d[r] = 1.0 - acc;
    }
    __syncthreads();
    const int best = block_argmax(d, m, false, red, redi);
    for (int r = tid; r < m; r += nt) u[r] = r == best ? 1.0 : 0.0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
        for (int q = tid; q < nq; q += nt) {
            const T* w = Q + (int64_t)q * m;
            double acc = 0.0;
            for (int r = 0; r < m; ++r) acc = fma(ld_fresh(w + r), u[r], acc);
            d[q] = acc;
        }
        __syncthreads();
        for (int r = tid; r < m; r += nt) {
            double acc = u[r];
            for (int q = 0; q < nq; ++q) acc = fma(-ld_fresh(Q + (int64_t)q * m + r), d[q], acc);
            u[r] = acc;
        }
        __syncthreads();
    }
    double nn = 0.0;
    for (int r = tid; r < m; r += nt) nn = fma(u[r], u[r], nn);
    const double inv = 1.0 / sqrt(block_sum_d(nn, red));
    for (int r = tid; r < m; r += nt) u[r] *= inv;
    __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(256) void k_tsvd_complete(TsvdCompleteArgs a) {
    __shared__ double u[kMaxRows], d[kMaxRows], red[4];
    __shared__ int redi[4];
    const int k = blockIdx.x, m = a.m, p = a.p, tid = threadIdx.x;
    T* Q = (T*)a.Lt + (int64_t)k * a.lt_ss;
    T* R = (T*)a.Rt + (int64_t)k * a.rt_ss;
    const double* sig = a.sig + (int64_t)k * a.sig_ss;
    // zero singular values: sorted after the nonzero ones, in column order
    int nz = 0;
    for (int c = 0; c < p; ++c) nz += sig[c] > 0.0 ? 1 : 0;
    int zc = -1;  // the original column of the current zero position
    for (int pos = nz; pos < p; ++pos) {
        for (zc = zc + 1; zc < p && sig[zc] > 0.0; ++zc) {
        }
        complement_vector<T>(Q, m, pos, u, d, red, redi);
        double f = 1.0;
        if (!a.sign_from_v) {
            // the pair's sign from the completed left vector itself
            const int bi = block_argmax(u, m, true, red, redi);
            if (u[bi] < 0.0) {
                f = -1.0;
                for (int r = tid; r < p; r += blockDim.x) R[(int64_t)pos * p + r] = -R[(int64_t)pos * p + r];
            }
        } else {
            // the pair's sign was taken from the Jacobi right vector (the left
            // vector of the wide slice) and already applied to it: apply it here
            const T* vj = (const T*)a.Vj + (int64_t)k * a.v_ss + (int64_t)zc * p;
            for (int r = tid; r < p; r += blockDim.x) d[r] = (double)vj[r];
            __syncthreads();
            const int bi = block_argmax(d, p, true, red, redi);
            if (d[bi] < 0.0) f = -1.0;
        }
        for (int r = tid; r < m; r += blockDim.x) Q[(int64_t)pos * m + r] = (T)(f * u[r]);
        __syncthreads();
    }
    if (!a.full) return;
    for (int c = p; c < m; ++c) {
        complement_vector<T>(Q, m, c, u, d, red, redi);
        const int bi = block_argmax(u, m, true, red, redi);
        const double f = u[bi] < 0.0 ? -1.0 : 1.0;
        for (int r = tid; r < m; r += blockDim.x) Q[(int64_t)c * m + r] = (T)(f * u[r]);
        __syncthreads();
    }
}

hipError_t launch_tsvd_complete(int prec, const TsvdCompleteArgs& a, hipStream_t s) {
    if (a.n3 <= 0) return hipSuccess;
    if (prec == 0) hipLaunchKernelGGL(k_tsvd_complete<double>, dim3(a.n3), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_tsvd_complete<float>, dim3(a.n3), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_tsvd_finish(int prec, const TsvdFinishArgs& a, hipStream_t s) {
    if (a.n3 <= 0) return hipSuccess;
    if (prec == 0) hipLaunchKernelGGL(k_tsvd_finish<double>, dim3(a.n3), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_tsvd_finish<float>, dim3(a.n3), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Utilities.  Zero-fill is a kernel (not a memset node) so it can sit in a
// captured graph.
// ---------------------------------------------------------------------------
// DFT path: slices of the real Fourier transform as real matrices.  The real
// transform puts the DC slice at 0, the real and imaginary parts of frequency
// f = 1..h at slots 2f-1 and 2f, and (even n3) the Nyquist slice at n3-1.  A
// complex slice B + iC is thresholded through its real form
//     E = [[B, -C], [C, B]]  (2 n1 x 2 n2),
// whose singular values are those of B + iC, each twice, and whose SVT at tau
// is the real form of the complex slice's SVT at tau.  embed writes E_f (f =
// 1..h, as slice f-1 of E) and the real slices (slice q of R); unembed takes
// B' = (E11 + E22) / 2 and C' = (E21 - E12) / 2 back to the slots.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void k_dft_embed(DftEmbedArgs a) {
    const int64_t n1 = a.n1, n2 = a.n2, s = n1 * n2;
    const int64_t ne = 4 * s * a.h, total = ne + s * a.nreal;
    const T* zb = (const T*)a.zb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < ne) {
            const int64_t f = e / (4 * s), o = e - f * 4 * s;
            const int64_t c = o / (2 * n1), r = o - c * 2 * n1;
            const int rb = r >= n1, cb = c >= n2;
            const int64_t i = r - rb * n1, j = c - cb * n2;
            const T* re = zb + (2 * f + 1) * s;
            const T* im = re + s;
            T v;
            if (rb == cb) v = re[i + n1 * j];
            else v = cb ? -im[i + n1 * j] : im[i + n1 * j];
            ((T*)a.E)[e] = v;
        } else {
            const int64_t q = (e - ne) / s, o = (e - ne) - q * s;
            const int64_t slot = q == 0 ? 0 : a.n3 - 1;
            ((T*)a.R)[e - ne] = zb[slot * s + o];
        }
    }
}

template <typename T>
__global__ void k_dft_unembed(DftEmbedArgs a) {
    const int64_t n1 = a.n1, n2 = a.n2, s = n1 * n2;
    const int64_t ne = 2 * s * a.h, total = ne + s * a.nreal;
    T* yb = (T*)a.zb;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (e < ne) {
            const int64_t f = e / (2 * s), o = e - f * 2 * s;
            const int part = o >= s;  // 0: real part, 1: imaginary part
            const int64_t ij = o - part * s, j = ij / n1, i = ij - j * n1;
            const T* E = (const T*)a.E + f * 4 * s;
            const int64_t ld = 2 * n1;
            T v;
            if (!part) v = (E[i + ld * j] + E[(n1 + i) + ld * (n2 + j)]) * (T)0.5;
            else v = (E[(n1 + i) + ld * j] - E[i + ld * (n2 + j)]) * (T)0.5;
            yb[(2 * f + 1 + part) * s + ij] = v;
        } else {
            const int64_t q = (e - ne) / s, o = (e - ne) - q * s;
            const int64_t slot = q == 0 ? 0 : a.n3 - 1;
            yb[slot * s + o] = ((const T*)a.R)[e - ne];
        }
    }
}

static unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

hipError_t launch_dft_embed(int prec, const DftEmbedArgs& a, hipStream_t s) {
    const int64_t total = a.n1 * a.n2 * (4 * (int64_t)a.h + a.nreal);
    if (prec == 0) hipLaunchKernelGGL(k_dft_embed<double>, dim3(grid_for(total)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_dft_embed<float>, dim3(grid_for(total)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_dft_unembed(int prec, const DftEmbedArgs& a, hipStream_t s) {
    const int64_t total = a.n1 * a.n2 * (2 * (int64_t)a.h + a.nreal);
    if (prec == 0) hipLaunchKernelGGL(k_dft_unembed<double>, dim3(grid_for(total)), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_dft_unembed<float>, dim3(grid_for(total)), dim3(256), 0, s, a);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void k_fill_zero(uint32_t* p, int64_t words) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_fill_zero(void* p, int64_t bytes, hipStream_t s) {
    const int64_t words = (bytes + 3) / 4;
    if (words <= 0) return hipSuccess;
    int64_t blocks = (words + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)blocks), dim3(256), 0, s, (uint32_t*)p, words);
    return hipGetLastError();
}

// Deterministic test pattern in [-1, 1): a 32-bit integer hash of (index,
// seed) (the "lowbias32" mixer: xorshift-multiply rounds), top 24 bits scaled.
__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

template <typename T>
__global__ void k_fill_pattern(T* p, int64_t n, uint32_t seed) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const uint32_t h = mix32((uint32_t)i ^ mix32(seed + (uint32_t)(i >> 32)));
        p[i] = (T)((double)(h >> 8) * (1.0 / 8388608.0) - 1.0);
    }
}

hipError_t launch_fill_pattern(void* p, int64_t n, int prec, uint32_t seed, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (prec == 0) hipLaunchKernelGGL(k_fill_pattern<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)p, n, seed);
    else hipLaunchKernelGGL(k_fill_pattern<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)p, n, seed);
    return hipGetLastError();
}

// Warm start of the completion's Jacobi SVDs: at iterations whose index (the
// device iteration counter) is a multiple of `period`, V of every slice is
// reset to the identity, which bounds the drift of V from orthogonality.
template <typename T>
__global__ void k_warm_reset(T* V, int p, int64_t total, const Ctrl* ctrl, int period) {
    if (ctrl->iter % period != 0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int64_t rc = e % ((int64_t)p * p);
        const int r = (int)(rc % p), c = (int)(rc / p);
        V[e] = (T)(r == c ? 1 : 0);
    }
}

hipError_t launch_warm_reset(int prec, void* V, int p, int n3, const Ctrl* ctrl, int period, hipStream_t s) {
    const int64_t total = (int64_t)p * p * n3;
    int64_t blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (prec == 0)
        hipLaunchKernelGGL(k_warm_reset<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)V, p, total, ctrl,
                           period);
    else
        hipLaunchKernelGGL(k_warm_reset<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)V, p, total, ctrl,
                           period);
    return hipGetLastError();
}

// End of one completion iteration: record the relative change in the history
// ring (slot iter mod hist_len), clear the norm accumulators, advance the
// iteration counter.
__global__ void k_iter_advance(Ctrl* ctrl, double* norms, double* hist, int hist_len) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double dn = 0.0, xn = 0.0;
        for (int i = 0; i < kNormSlots; ++i) {
            dn += norms[2 * i];
            xn += norms[2 * i + 1];
            norms[2 * i] = 0.0;
            norms[2 * i + 1] = 0.0;
        }
        const double rc = xn > 0.0 ? sqrt(dn / xn) : sqrt(dn);
        const int it = ctrl->iter;
        hist[it % hist_len] = rc;
        ctrl->iter = it + 1;
    }
}

hipError_t launch_iter_advance(Ctrl* ctrl, double* norms, double* relchg_hist, int hist_len, hipStream_t s) {
    hipLaunchKernelGGL(k_iter_advance, dim3(1), dim3(64), 0, s, ctrl, norms, relchg_hist, hist_len);
    return hipGetLastError();
}

// Algorithm 1's initial iterate: X = B on the observed set, 0 elsewhere.
template <typename T>
__global__ void k_observed_init(T* X, const T* B, const uint8_t* mask, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride)
        X[e] = mask[e] ? B[e] : (T)0;
}

hipError_t launch_observed_init(int prec, void* X, const void* B, const uint8_t* mask, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (prec == 0)
        hipLaunchKernelGGL(k_observed_init<double>, dim3((unsigned)blocks), dim3(256), 0, s, (double*)X,
                           (const double*)B, mask, n);
    else
        hipLaunchKernelGGL(k_observed_init<float>, dim3((unsigned)blocks), dim3(256), 0, s, (float*)X,
                           (const float*)B, mask, n);
    return hipGetLastError();
}

// Per-job control blocks of a batched step folded into the launch's block:
// status bits ORed, largest sweep count and summed slice-sweeps.
__global__ void k_fold_ctrl(Ctrl* dst, const Ctrl* jobs, int count, int stride_bytes) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int st = 0, ms = 0;
    unsigned long long sw = 0;
    for (int j = 0; j < count; ++j) {
        const Ctrl* c = (const Ctrl*)((const char*)jobs + (int64_t)j * stride_bytes);
        st |= c->status;
        ms = c->max_sweeps > ms ? c->max_sweeps : ms;
        sw += c->slice_sweeps;
    }
    dst->status |= st;
    if (ms > dst->max_sweeps) dst->max_sweeps = ms;
    dst->slice_sweeps += sw;
}

hipError_t launch_fold_ctrl(Ctrl* dst, const Ctrl* jobs, int count, int stride_bytes, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fold_ctrl, dim3(1), dim3(64), 0, s, dst, jobs, count, stride_bytes);
    return hipGetLastError();
}

}  // namespace tsvd
