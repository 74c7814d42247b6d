// Threshold certificate of the kept-column Jacobi mode.
//
// Singular value thresholding (Theorem 5) keeps only the singular values
// above tau and their vectors, so the one-sided Jacobi iteration of a t-SVT
// slice may stop once the columns that carry them are settled.  The kept-
// column mode (jacobi.hip) leaves a slice's work matrix A' = A W (W
// orthogonal) with columns K of squared norm > tau^2 and the rest R, every
// column of K orthogonal to every other column of A' -- to the iteration's
// own convergence test, the evidence the full iteration rests on as well
// (the mode never rotates two columns of R, so nothing stirs K against R
// after its pairs were checked).  Then the singular values of A are the
// norms of K's columns together with R's singular values, and if
//   the spectral norm of R is at most tau,
// the thresholding keeps exactly the columns of K above tau, which is what
// the rebuild uses.  That is the one fact the iteration cannot see, and the
// certificate checks it: with H = R^T R / tau^2 (symmetric, positive
// semidefinite),
//   (sigma_max(R) / tau)^16 = lambda_max(H)^8 <= trace(H^8) = ||H^4||_F^2,
// a bound that is tight when few singular values of R are near its largest.
// H^4 takes two squarings; everything from the Gram matrix on is FP32 on
// A' / tau, with a rounding margin (below) that the test must clear.
//
// A slice that fails, or whose kept-column iteration did not converge, is
// marked for the full Jacobi iteration, which the caller then runs from A'
// (a slice that passes is left alone by that launch).  A slice that the
// kept-column iteration already finished as the full iteration passes as it
// is.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.h"

namespace tsvd {
namespace {

constexpr int kCertThreads = 256;  // four wavefronts, one column each
constexpr int kCertRows = kMaxRows / kWave;  // rows per lane (m <= kMaxRows)

__device__ __forceinline__ double cert_tau(const CertArgs& a) {
    return a.tau_sched ? a.tau_sched[a.ctrl->iter] : a.tau;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// One wavefront per column: its squared norm in FP64, and the column scaled
// by 1/tau as FP32 (the Gram operand), or zero for a kept column (squared
// norm > tau^2), so that the Gram matrix is H with the kept columns' rows and
// columns zero.  Slices that converged as the full iteration are skipped
// (GEMM column count 0, verdict 1).
template <typename T>
__global__ __launch_bounds__(kCertThreads) void k_cert_scan(CertArgs a) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t col = (int64_t)blockIdx.x * (kCertThreads / kWave) + wave;
    if (col >= (int64_t)a.n3 * a.p) return;
    const int k = (int)(col / a.p);
    const bool skip = a.full[k] != 0;
    if (lane == 0 && col - (int64_t)k * a.p == 0) {
        a.ncols[k] = skip ? 0 : a.p;
        a.flags[k] = skip ? 1 : 0;
    }
    if (skip) return;
    const T* x = (const T*)a.A + col * a.m;
    float* y = a.As + col * a.m;
    double v[kCertRows];
    double acc = 0.0;
#pragma unroll
    for (int q = 0; q < kCertRows; ++q) {
        const int r = lane + kWave * q;
        v[q] = r < a.m ? (double)x[r] : 0.0;
        acc = fma(v[q], v[q], acc);
    }
    acc = wave_sum_d(acc);
    if (lane == 0) a.nrm2[col] = acc;
    const double tau = cert_tau(a);
    const bool kept = acc > tau * tau;  // (a NaN norm stays in H and fails the test)
    const double inv = 1.0 / tau;
#pragma unroll
    for (int q = 0; q < kCertRows; ++q) {
        const int r = lane + kWave * q;
        if (r < a.m) y[r] = kept ? 0.0f : (float)(v[q] * inv);
    }
}

// ||H^4||_F^2 per slice and the verdict: grid (chunks, slices); each
// workgroup adds its FP64 partial sum to sums[k] (zero before the launch),
// and the last one of a slice to finish decides.  The margin covers the FP32
// Gram matrix (entrywise error <= gamma_m |R|^T |R| / tau^2, whose spectral
// norm is at most gamma_m trace(H)) and the two squarings:
//   delta = 2 (m + 2 p) u32 trace(H) + 2^-8,  pass iff ||H^4||_F^2 <= (1 - delta)^8.
__global__ __launch_bounds__(kCertThreads) void k_cert_verdict(CertArgs a) {
    __shared__ double s_part[kCertThreads / kWave];
    __shared__ int s_last;
    const int k = blockIdx.y, tid = threadIdx.x;
    if (a.full[k]) return;  // (the same for the whole workgroup; the scan set its verdict)
    const int64_t pp = (int64_t)a.p * a.p;
    const float* H4 = a.H + (int64_t)k * pp;
    double s = 0.0;
    for (int64_t e = (int64_t)blockIdx.x * kCertThreads + tid; e < pp; e += (int64_t)gridDim.x * kCertThreads) {
        const double v = (double)H4[e];
        s = fma(v, v, s);
    }
    s = wave_sum_d(s);
    if ((tid & 63) == 0) s_part[tid >> 6] = s;
    __syncthreads();
    if (tid == 0) {
        double S = 0.0;
        for (int w = 0; w < kCertThreads / kWave; ++w) S += s_part[w];
        atomicAdd(a.sums + k, S);
        __threadfence();
        s_last = atomicAdd(a.done + k, 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (!s_last) return;
    // the slice's last workgroup: every partial sum is in sums[k]
    const double* nk = a.nrm2 + (int64_t)k * a.p;
    const double tau = cert_tau(a), t2 = tau * tau;
    double tr = 0.0;
    for (int c = tid; c < a.p; c += kCertThreads)
        if (!(nk[c] > t2)) tr += nk[c] / t2;
    tr = wave_sum_d(tr);
    __syncthreads();  // s_part is reused
    if ((tid & 63) == 0) s_part[tid >> 6] = tr;
    __syncthreads();
    if (tid == 0) {
        double TR = 0.0;
        for (int w = 0; w < kCertThreads / kWave; ++w) TR += s_part[w];
        const double S = __hip_atomic_load(a.sums + k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const double delta = 2.0 * (a.m + 2.0 * a.p) * 0x1p-24 * TR + 0x1p-8;
        const double b = 1.0 - delta, b2 = b * b, b4 = b2 * b2;
        const bool ok = a.sweeps[k] >= 0 && delta < 1.0 && S <= b4 * b4;
        a.flags[k] = ok ? 1 : 0;
        if (!ok) atomicAdd(&a.ctrl->fallback, 1);
    }
}

}  // namespace

hipError_t launch_threshold_certificate(int prec, CertArgs a, hipStream_t s) {
    if (a.n3 <= 0 || a.p <= 0) return hipSuccess;
    if (a.m > kMaxRows || (!a.tau_sched && !(a.tau > 0.0))) return hipErrorInvalidValue;
    const int64_t cols = (int64_t)a.n3 * a.p;
    const dim3 gcols((unsigned)((cols + 3) / 4)), blk(kCertThreads);
    if (prec == 0) hipLaunchKernelGGL(k_cert_scan<double>, gcols, blk, 0, s, a);
    else hipLaunchKernelGGL(k_cert_scan<float>, gcols, blk, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t pp = (int64_t)a.p * a.p;
    // Gram matrix of A' / tau: G = As^T As
    GemmArgs g{};
    g.A = a.As; g.a_rs = a.m; g.a_cs = 1; g.a_bs = (int64_t)a.m * a.p;
    g.B = a.As; g.b_rs = 1; g.b_cs = a.m; g.b_bs = (int64_t)a.m * a.p;
    g.C = a.H; g.c_rs = 1; g.c_cs = a.p; g.c_bs = pp;
    g.M = a.p; g.Nn = a.p; g.K = a.m; g.batch = a.n3;
    g.Ndev = a.ncols;
    if ((e = launch_gemm(1, g, s)) != hipSuccess) return e;
    // H^2 into H2, then H^4 back into H
    GemmArgs q{};
    q.a_rs = 1; q.a_cs = a.p; q.a_bs = pp;
    q.b_rs = 1; q.b_cs = a.p; q.b_bs = pp;
    q.c_rs = 1; q.c_cs = a.p; q.c_bs = pp;
    q.M = a.p; q.Nn = a.p; q.K = a.p; q.batch = a.n3;
    q.Ndev = a.ncols;
    q.A = a.H; q.B = a.H; q.C = a.H2;
    if ((e = launch_gemm(1, q, s)) != hipSuccess) return e;
    q.A = a.H2; q.B = a.H2; q.C = a.H;
    if ((e = launch_gemm(1, q, s)) != hipSuccess) return e;
    const unsigned chunks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(16, pp / (8 * kCertThreads)));
    hipLaunchKernelGGL(k_cert_verdict, dim3(chunks, (unsigned)a.n3), blk, 0, s, a);
    return hipGetLastError();
}

}  // namespace tsvd
