// Fast tube transforms for long tubes: the orthonormal DCT-II along every
// tube (Section 3, dct(.,[],3)) and its inverse in O(n3 log n3) work, for
// tubes longer than the matrix-core kernel's limit.
//
// Forward (Makhoul's reordering): with v[t] = x[2t] for t < ceil(n/2) and
// v[n-1-t] = x[2t+1] for t < floor(n/2), the unnormalized DCT-II is
//     y[k] = sum_t x[t] cos(pi (2t+1) k / (2n)) = Re(e^{-i pi k/(2n)} V[k]),
// V = DFT_n(v), and X[k] = s_k y[k] (s_0 = sqrt(1/n), s_k = sqrt(2/n)).
// Inverse: y[k] = X[k] / s_k, V[k] = e^{i pi k/(2n)} (y[k] - i y[n-k])
// (y[n] = 0), v = IDFT_n(V) (real), x[2t] = v[t], x[2t+1] = v[n-1-t].
//
// DFT_n of any length by Bluestein's chirp: with c[j] = e^{-i pi j^2 / n},
// DFT_n(u)[k] = c[k] sum_j (u[j] c[j]) conj(c[k-j]), a linear convolution
// done as a cyclic one of length M (a power of two >= 2n - 1): a forward
// radix-2 FFT of the chirped input (decimation in frequency: natural order
// in, bit-reversed order out), a product with the transformed conjugate chirp
// (stored bit-reversed on the host), and an inverse radix-2 FFT (decimation
// in time: bit-reversed order in, natural order out), so that no explicit
// permutation is needed.  The inverse DFT is conj(DFT_n(conj(V))) / n.
//
// Workgroup: 16 consecutive tubes (each row of the mode-3 unfolding read and
// written as 16-element runs), staged in LDS; each of the 4 wavefronts takes
// tubes w, w+4, w+8, w+12 in turn, with an M-point complex FP64 buffer of its
// own.  The completion prologue and epilogue are applied as in the dense
// kernels.  All arithmetic is FP64; tables (twiddles, chirps, the transformed
// chirp, the DCT phases) are FP64 and built on the host.
//
// The same kernel computes the real form of the DFT along the tubes (the
// Fourier-domain t-SVD of Section 2): row 0 = Re V[0], rows 2f - 1 and 2f =
// Re V[f] and Im V[f] for 1 <= f <= (n - 1) / 2, and for even n row n - 1 =
// V[n/2] (real), V = DFT_n(x); its inverse rebuilds the Hermitian spectrum and
// returns Re IDFT_n.
#include <math.h>

#include <complex>
#include <vector>

#include "internal.h"

namespace tsvd {

constexpr int kFftTubes = 16;
constexpr int kFftLd = kFftTubes + 1;  // LDS row pitch of the tube tile (odd: no bank conflicts down a tube)

// Orders the LDS accesses of one wavefront (the hardware keeps them in order;
// this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct FftTables {
    const double2* tw;     // M/2: e^{-2 pi i j / M}
    const double2* chirp;  // n: c[j] = e^{-i pi j^2 / n}
    const double2* bhat;   // M: FFT_M of the wrapped conjugate chirp, bit-reversed order
    const double2* phase;  // n: e^{-i pi k / (2n)}
    int n, M, logM;
};

// Bytes of the tube tile, rounded up to 16 so that the FFT buffers after it are aligned.
__host__ __device__ __forceinline__ int fft_tile_bytes(int n) { return (n * kFftLd * 8 + 15) & ~15; }

__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cconj(double2 a) { return make_double2(a.x, -a.y); }

// In-place radix-2 FFT of M points in LDS by one wavefront.  dif: forward
// decimation in frequency (natural in, bit-reversed out, twiddles e^{-}); else
// decimation in time with conjugate twiddles (bit-reversed in, natural out):
// the unscaled inverse.  LDS accesses of one wavefront complete in program
// order, so the stages need no workgroup barrier.
__device__ void fft_wave(double2* buf, const FftTables& t, bool dif) {
    const int lane = threadIdx.x & 63, M = t.M;
    for (int s = 0; s < t.logM; ++s) {
        const int h = dif ? (M >> (s + 1)) : (1 << s);  // half-size of the butterflies
        const int stride = M / (2 * h);                  // twiddle stride in tw
        for (int b = lane; b < M / 2; b += 64) {
            const int grp = b / h, j = b - grp * h;
            const int i0 = grp * 2 * h + j, i1 = i0 + h;
            double2 w = t.tw[j * stride];
            const double2 x0 = buf[i0], x1 = buf[i1];
            if (dif) {
                buf[i0] = make_double2(x0.x + x1.x, x0.y + x1.y);
                buf[i1] = cmul(make_double2(x0.x - x1.x, x0.y - x1.y), w);
            } else {
                w = cconj(w);
                const double2 y = cmul(x1, w);
                buf[i0] = make_double2(x0.x + y.x, x0.y + y.y);
                buf[i1] = make_double2(x0.x - y.x, x0.y - y.y);
            }
        }
        wave_sync();
    }
}

// DFT_n of u (n values in buf[0..n)) into buf[0..n), by the chirp.
__device__ void dft_bluestein(double2* buf, const FftTables& t) {
    const int lane = threadIdx.x & 63;
    for (int j = lane; j < t.M; j += 64) buf[j] = j < t.n ? cmul(buf[j], t.chirp[j]) : make_double2(0.0, 0.0);
    wave_sync();
    fft_wave(buf, t, true);
    for (int j = lane; j < t.M; j += 64) buf[j] = cmul(buf[j], t.bhat[j]);
    wave_sync();
    fft_wave(buf, t, false);
    const double inv = 1.0 / t.M;
    for (int k = lane; k < t.n; k += 64) {
        const double2 v = cmul(buf[k], t.chirp[k]);
        buf[k] = make_double2(v.x * inv, v.y * inv);
    }
    wave_sync();
}

template <typename T>
__global__ __launch_bounds__(256) void k_tube_fft(TubeArgs a, FftTables t, int mode) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double s_red[2][4];
    const int n = a.n3, M = t.M;
    const int64_t N = a.N;
    double* tile = (double*)smem_raw;                              // n rows of 16 tubes, pitch kFftLd
    double2* bufs = (double2*)(smem_raw + fft_tile_bytes(n));      // 4 x M
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.x * kFftTubes;
    double beta = 1.0;
    if (a.pX || a.eX) beta = a.beta_sched ? a.beta_sched[a.ctrl->iter] : a.beta_val;

    // load: element (tube q, position k) -> tile[k * kFftLd + q], 16-element runs
    int bad = 0;
    for (int e = tid; e < n * kFftTubes; e += 256) {
        const int k = e / kFftTubes, q = e - k * kFftTubes;
        const int64_t r = r0 + q;
        double v = 0.0;
        if (r < N) {
            const int64_t g = r + N * k;
            if (a.pX) v = (double)((const T*)a.pX)[g] - (double)((const T*)a.pM)[g] / beta;
            else v = (double)((const T*)a.in)[g];
            v = (double)(T)v;  // the value the dense kernels see
            if (a.check_finite && !isfinite(v)) bad = 1;
        }
        tile[k * kFftLd + q] = v;
    }
    if (a.check_finite && bad) atomicOr(&a.ctrl->status, kStNonFinite);
    __syncthreads();

    double2* buf = bufs + (size_t)wave * M;
    const double s0 = sqrt(1.0 / n), s1 = sqrt(2.0 / n);
    for (int q = wave; q < kFftTubes; q += 4) {
        if (r0 + q >= N) break;
        if (mode == kFftDftForward) {
            for (int j = lane; j < n; j += 64) buf[j] = make_double2(tile[j * kFftLd + q], 0.0);
            wave_sync();
            dft_bluestein(buf, t);
            for (int k = lane; k < n; k += 64) {
                double y;
                if (k == 0) y = buf[0].x;
                else if ((n & 1) == 0 && k == n - 1) y = buf[n / 2].x;
                else y = (k & 1) ? buf[(k + 1) / 2].x : buf[k / 2].y;
                tile[k * kFftLd + q] = y;
            }
        } else if (mode == kFftDftInverse) {
            // conj(V) of the Hermitian spectrum; x = Re DFT(conj V) / n
            const int h = (n - 1) / 2;
            for (int k = lane; k < n; k += 64) {
                double re, im;
                if (k == 0) { re = tile[q]; im = 0.0; }
                else if ((n & 1) == 0 && k == n / 2) { re = tile[(n - 1) * kFftLd + q]; im = 0.0; }
                else if (k <= h) { re = tile[(2 * k - 1) * kFftLd + q]; im = tile[2 * k * kFftLd + q]; }
                else { re = tile[(2 * (n - k) - 1) * kFftLd + q]; im = -tile[2 * (n - k) * kFftLd + q]; }
                buf[k] = make_double2(re, -im);
            }
            wave_sync();
            dft_bluestein(buf, t);
            for (int j = lane; j < n; j += 64) tile[j * kFftLd + q] = buf[j].x / n;
        } else if (mode == kFftDctForward) {
            // v[t] = x[2t], v[n-1-t] = x[2t+1]
            for (int j = lane; j < n; j += 64) {
                const int src = (2 * j < n) ? 2 * j : 2 * (n - 1 - j) + 1;
                buf[j] = make_double2(tile[src * kFftLd + q], 0.0);
            }
            wave_sync();
            dft_bluestein(buf, t);
            for (int k = lane; k < n; k += 64) {
                const double2 z = cmul(t.phase[k], buf[k]);
                tile[k * kFftLd + q] = (k == 0 ? s0 : s1) * z.x;
            }
        } else {
            // V[k] = e^{i pi k/(2n)} (y[k] - i y[n-k]), y = X / s; the inverse DFT as
            // conj(DFT(conj(V))) / n, so the input is conj(V)
            for (int k = lane; k < n; k += 64) {
                const double yk = tile[k * kFftLd + q] / (k == 0 ? s0 : s1);
                const double ynk = k == 0 ? 0.0 : tile[(n - k) * kFftLd + q] / s1;
                const double2 v = cmul(cconj(t.phase[k]), make_double2(yk, -ynk));
                buf[k] = cconj(v);
            }
            wave_sync();
            dft_bluestein(buf, t);
            // x[2t] = v[t], x[2t+1] = v[n-1-t] with v = conj(DFT(...)) / n (real part)
            for (int j = lane; j < n; j += 64) {
                const int dst = (2 * j < n) ? 2 * j : 2 * (n - 1 - j) + 1;
                tile[dst * kFftLd + q] = buf[j].x / n;
            }
        }
        wave_sync();
    }
    __syncthreads();

    // store (and the completion epilogue), 16-element runs
    double dn = 0.0, xn = 0.0;
    for (int e = tid; e < n * kFftTubes; e += 256) {
        const int k = e / kFftTubes, q = e - k * kFftTubes;
        const int64_t r = r0 + q;
        if (r >= N) continue;
        const int64_t g = r + N * k;
        const T y = (T)tile[k * kFftLd + q];
        if (a.out) ((T*)a.out)[g] = y;
        if (a.eX) {
            T* X = (T*)a.eX;
            T* Ml = (T*)a.eM;
            const T xold = X[g];
            const T mold = Ml[g];
            T xnew;
            if (a.emask[g]) xnew = ((const T*)a.eB)[g];
            else xnew = (T)((double)y + (double)mold / beta);
            Ml[g] = (T)((double)mold + beta * ((double)y - (double)xnew));
            X[g] = xnew;
            const double d = (double)xnew - (double)xold;
            dn += d * d;
            xn += (double)xold * (double)xold;
        }
    }
    if (a.eX && a.norms) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            dn += __shfl_xor(dn, o, kWave);
            xn += __shfl_xor(xn, o, kWave);
        }
        if (lane == 0) {
            s_red[0][wave] = dn;
            s_red[1][wave] = xn;
        }
        __syncthreads();
        if (tid == 0) {
            double* slot = a.norms + 2 * (blockIdx.x % kNormSlots);
            atomicAdd(slot, s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3]);
            atomicAdd(slot + 1, s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3]);
        }
    }
}

// ---- host side ------------------------------------------------------------------

int fft_size(int n) {
    int M = 1;
    while (M < 2 * n - 1) M <<= 1;
    return M;
}

size_t fft_table_bytes(int n) {
    const int M = fft_size(n);
    return sizeof(double) * 2 * ((size_t)M / 2 + n + M + n);
}

static int bit_reverse(int x, int bits) {
    int y = 0;
    for (int b = 0; b < bits; ++b) y |= ((x >> b) & 1) << (bits - 1 - b);
    return y;
}

// Tables in FP64: twiddles e^{-2 pi i j/M}; chirp c[j] = e^{-i pi (j^2 mod 2n)/n};
// the transformed wrapped conjugate chirp (an O(M^2) DFT in long double, once
// per length), stored bit-reversed; DCT phases e^{-i pi k/(2n)}.
void make_fft_tables(int n, void* out) {
    const int M = fft_size(n);
    int logM = 0;
    while ((1 << logM) < M) ++logM;
    const long double pi = acosl(-1.0L);
    double* p = (double*)out;
    double* tw = p;
    double* ch = tw + M;       // M/2 complex
    double* bh = ch + 2 * n;   // n complex
    double* ph = bh + 2 * M;   // M complex
    for (int j = 0; j < M / 2; ++j) {
        const long double ang = -2.0L * pi * j / M;
        tw[2 * j] = (double)cosl(ang);
        tw[2 * j + 1] = (double)sinl(ang);
    }
    std::vector<std::complex<long double>> c(n), b(M, 0.0L);
    for (int j = 0; j < n; ++j) {
        const long long q = ((long long)j * j) % (2LL * n);
        const long double ang = -pi * (long double)q / n;
        c[j] = std::complex<long double>(cosl(ang), sinl(ang));
        ch[2 * j] = (double)c[j].real();
        ch[2 * j + 1] = (double)c[j].imag();
    }
    // wrapped conj(c): b[m] = conj(c[m]) for m < n, b[M - m] = conj(c[m]) for 0 < m < n
    for (int m = 0; m < n; ++m) {
        b[m] = std::conj(c[m]);
        if (m > 0) b[M - m] = std::conj(c[m]);
    }
    for (int k = 0; k < M; ++k) {
        std::complex<long double> acc = 0.0L;
        for (int m = 0; m < M; ++m) {
            if (b[m] == std::complex<long double>(0.0L, 0.0L)) continue;
            const long long q = ((long long)k * m) % M;
            const long double ang = -2.0L * pi * (long double)q / M;
            acc += b[m] * std::complex<long double>(cosl(ang), sinl(ang));
        }
        const int kr = bit_reverse(k, logM);
        bh[2 * kr] = (double)acc.real();
        bh[2 * kr + 1] = (double)acc.imag();
    }
    for (int k = 0; k < n; ++k) {
        const long double ang = -pi * k / (2.0L * n);
        ph[2 * k] = (double)cosl(ang);
        ph[2 * k + 1] = (double)sinl(ang);
    }
}

int fft_lds_bytes(int n) { return fft_tile_bytes(n) + 4 * fft_size(n) * 16; }

bool fft_fits(int n3) { return n3 > kMaxTube && fft_lds_bytes(n3) <= kLdsBudget; }

hipError_t launch_tube_fft(int prec, const TubeArgs& a, const void* tables, int mode, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    const int n = a.n3, M = fft_size(n);
    if (fft_lds_bytes(n) > kLdsBudget) return hipErrorInvalidValue;
    FftTables t;
    const double* p = (const double*)tables;
    t.tw = (const double2*)p;
    t.chirp = (const double2*)(p + M);
    t.bhat = (const double2*)(p + M + 2 * n);
    t.phase = (const double2*)(p + M + 2 * n + 2 * M);
    t.n = n;
    t.M = M;
    t.logM = 0;
    while ((1 << t.logM) < M) ++t.logM;
    const int lds = fft_lds_bytes(n);
    const dim3 grid((unsigned)((a.N + kFftTubes - 1) / kFftTubes)), block(256);
    const void* f = prec == 0 ? (const void*)k_tube_fft<double> : (const void*)k_tube_fft<float>;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    if (prec == 0) hipLaunchKernelGGL(k_tube_fft<double>, grid, block, lds, s, a, t, mode);
    else hipLaunchKernelGGL(k_tube_fft<float>, grid, block, lds, s, a, t, mode);
    return hipGetLastError();
}

}  // namespace tsvd
