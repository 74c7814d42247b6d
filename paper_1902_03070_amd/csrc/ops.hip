// Tube transforms, batched slice GEMMs and the thresholding step.
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
constexpr int kTubeTile = 64;
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
            atomicAdd(&a.norms[0], s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3]);
            atomicAdd(&a.norms[1], s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3]);
        }
    }
}

hipError_t launch_tube_transform(int prec, const TubeArgs& a, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    dim3 grid((unsigned)((a.N + kTubeTile - 1) / kTubeTile)), block(256);
    if (prec == 0) {
        const int lds = a.n3 * kTubeTile * 8;
        hipLaunchKernelGGL(k_tube<double>, grid, block, lds, s, a);
    } else {
        const int lds = a.n3 * kTubeTile * 4;
        hipLaunchKernelGGL(k_tube<float>, grid, block, lds, s, a);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Batched strided GEMM  C_b = (A_b B_b) diag(cscale_b), K_b from Kdev or K.
// 64 x 64 output tile per workgroup, 256 threads, 4 x 4 outputs per thread
// (rows tx + 16u, columns ty + 16v), K staged through LDS in chunks of 16.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g) {
    __shared__ T As[16][64 + 1];
    __shared__ T Bs[16][64 + 1];
    const int b = blockIdx.z;
    const int i0 = blockIdx.x * 64, j0 = blockIdx.y * 64;
    const int K = g.Kdev ? g.Kdev[b] : g.K;
    const int Nb = g.Ndev ? g.Ndev[b] : g.Nn;
    if (j0 >= Nb) return;
    const int tid = threadIdx.x, tx = tid % 16, ty = tid / 16;
    const T* A = (const T*)g.A + (int64_t)b * g.a_bs;
    const T* B = (const T*)g.B + (int64_t)b * g.b_bs;
    T acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = (T)0;
    const bool a_rowfast = g.a_rs == 1;
    const bool b_rowfast = g.b_rs == 1;
    for (int t0 = 0; t0 < K; t0 += 16) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int e = tid + 256 * q;
            int ii, tt;
            if (a_rowfast) { ii = e % 64; tt = e / 64; }
            else { tt = e % 16; ii = e / 16; }
            const int gi = i0 + ii, gt = t0 + tt;
            As[tt][ii] = (gi < g.M && gt < K) ? A[(int64_t)gi * g.a_rs + (int64_t)gt * g.a_cs] : (T)0;
            int jj;
            if (b_rowfast) { tt = e % 16; jj = e / 16; }
            else { jj = e % 64; tt = e / 64; }
            const int gj = j0 + jj, gt2 = t0 + tt;
            Bs[tt][jj] = (gj < Nb && gt2 < K) ? B[(int64_t)gt2 * g.b_rs + (int64_t)gj * g.b_cs] : (T)0;
        }
        __syncthreads();
#pragma unroll
        for (int tt = 0; tt < 16; ++tt) {
            T av[4], bv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) av[u] = As[tt][tx + 16 * u];
#pragma unroll
            for (int v = 0; v < 4; ++v) bv[v] = Bs[tt][ty + 16 * v];
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(av[u], bv[v], acc[u][v]);
        }
        __syncthreads();
    }
    T* C = (T*)g.C + (int64_t)b * g.c_bs;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int j = j0 + ty + 16 * v;
        if (j >= Nb) continue;
        const double sc = g.cscale ? g.cscale[(int64_t)b * g.s_bs + j] : 1.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = i0 + tx + 16 * u;
            if (i < g.M) C[(int64_t)i * g.c_rs + (int64_t)j * g.c_cs] = g.cscale ? (T)((double)acc[u][v] * sc) : acc[u][v];
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

// End of one completion iteration: record the relative change, clear the
// norm accumulators, advance the iteration counter.
__global__ void k_iter_advance(Ctrl* ctrl, double* norms, double* hist, int hist_len) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double dn = norms[0], xn = norms[1];
        const double rc = xn > 0.0 ? sqrt(dn / xn) : sqrt(dn);
        const int it = ctrl->iter;
        if (it < hist_len) hist[it] = rc;
        norms[0] = 0.0;
        norms[1] = 0.0;
        ctrl->iter = it + 1;
    }
}

hipError_t launch_iter_advance(Ctrl* ctrl, double* norms, double* relchg_hist, int hist_len, hipStream_t s) {
    hipLaunchKernelGGL(k_iter_advance, dim3(1), dim3(64), 0, s, ctrl, norms, relchg_hist, hist_len);
    return hipGetLastError();
}

}  // namespace tsvd
