// Fast tube transforms for long tubes: the orthonormal DCT-II along every
// tube (Section 3, dct(.,[],3)) and its inverse, and the real form of the DFT
// along the tubes (Section 2) and its inverse, in O(n3 log n3) work, for
// tubes longer than the matrix-core kernel's limit.
//
// DCT-II by Makhoul's reordering: with v[t] = x[2t] for t < ceil(n/2) and
// v[n-1-t] = x[2t+1] for t < floor(n/2), the unnormalized DCT-II is
//     y[k] = sum_t x[t] cos(pi (2t+1) k / (2n)) = Re(e^{-i pi k/(2n)} V[k]),
// V = DFT_n(v), and X[k] = s_k y[k] (s_0 = sqrt(1/n), s_k = sqrt(2/n)).
// Inverse: y[k] = X[k] / s_k, V[k] = e^{i pi k/(2n)} (y[k] - i y[n-k])
// (y[n] = 0), v = IDFT_n(V) (real), x[2t] = v[t], x[2t+1] = v[n-1-t].
//
// Real form of the DFT (the Fourier path's tube transform): row 0 = Re V[0],
// rows 2f - 1 and 2f = Re V[f] and Im V[f] for 1 <= f <= (n - 1) / 2, and
// for even n row n - 1 = V[n/2] (real), V = DFT_n(x); the inverse rebuilds the
// Hermitian spectrum and returns IDFT_n (real).
//
// Two real tubes per complex transform: the DFT of u = v1 + i v2 gives
// V1[k] = (W[k] + conj W[n-k]) / 2 and V2[k] = (W[k] - conj W[n-k]) / (2i);
// the inverse DFT of V1 + i V2 is v1 + i v2 when both are real.
//
// DFT_n of any length by Bluestein's chirp: with c[j] = e^{-i pi j^2 / n},
// DFT_n(u)[k] = c[k] sum_j (u[j] c[j]) conj(c[k-j]), a linear convolution
// done as a cyclic one of length M = 64 R (a power of two >= 2n - 1): an FFT
// of the chirped input, a product with the FFT of the wrapped conjugate chirp
// (a table), and an inverse FFT taken as conj(FFT(conj .)).  An inverse DFT is
// conj(DFT(conj .)) / n.
//
// FFT of M points by one wavefront, Stockham autosort (natural order in and
// out, no bit reversal): lane l holds x[l + 64 s], s < R, in registers; each
// pass of radix r applies the twiddles and r-point DFTs in registers and
// exchanges through LDS (three passes: 8 x 8 x 8 for M = 512, 16 x 16 x 4 for
// M = 1024).
//
// Workgroup: 16 consecutive tubes (each row of the mode-3 unfolding read and
// written as 16-element runs), staged in LDS in the data type; each of the 4
// wavefronts transforms tube pairs w and w + 4 with an M-point complex
// exchange buffer of its own.  The completion prologue and epilogue are
// applied as in the dense kernels.  The arithmetic and the tables (twiddles,
// chirp, transformed chirp, DCT phases; built on the host in long double) are
// FP64 for double data and FP32 for float data.
#include <math.h>

#include <complex>
#include <vector>

#include "internal.h"

namespace tsvd {

constexpr int kFftTubes = 16;
constexpr int kFftLd = kFftTubes + 1;  // LDS row pitch of the tube tile (odd: fewer bank conflicts down a tube)

// Complex value of the compute type C (double or float), aligned so that LDS
// and table accesses are single wide loads and stores.
template <typename C>
struct __align__(2 * sizeof(C)) cx {
    C x, y;
};

template <typename C>
struct FftTables {
    const cx<C>* tw;     // M: e^{-2 pi i t / M}
    const cx<C>* chirp;  // M: c[j] = e^{-i pi j^2 / n} for j < n, then zeros
    const cx<C>* bhat;   // M: FFT_M of the wrapped conjugate chirp
    const cx<C>* phase;  // M/2: e^{-i pi k / (2n)} for k < n, then zeros
    int n;
};

// Orders the LDS accesses of one wavefront (the hardware keeps them in order;
// this keeps the compiler from moving them across).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Tile bytes (data type es), rounded up to 16 so that the buffers after it are aligned.
__host__ __device__ __forceinline__ int fft_tile_bytes(int n, int es) { return (n * kFftLd * es + 15) & ~15; }
// Exchange buffer index: one pad slot per 16 entries against bank conflicts.
__host__ __device__ __forceinline__ int fpad(int i) { return i + (i >> 4); }
__host__ __device__ __forceinline__ int fft_buf_entries(int M) { return fpad(M - 1) + 1; }

template <typename C>
__device__ __forceinline__ cx<C> mkc(C x, C y) {
    cx<C> r;
    r.x = x;
    r.y = y;
    return r;
}
template <typename C>
__device__ __forceinline__ cx<C> cadd(cx<C> a, cx<C> b) { return mkc<C>(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ __forceinline__ cx<C> csub(cx<C> a, cx<C> b) { return mkc<C>(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ __forceinline__ cx<C> cmul(cx<C> a, cx<C> b) {
    return mkc<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C>
__device__ __forceinline__ cx<C> cconj(cx<C> a) { return mkc<C>(a.x, -a.y); }
template <typename C>
__device__ __forceinline__ cx<C> cscale(cx<C> a, C s) { return mkc<C>(a.x * s, a.y * s); }

// cos and sin of 2 pi m / 16
constexpr double kC1 = 0.92387953251128675613;  // cos(pi/8)
constexpr double kS1 = 0.38268343236508977173;  // sin(pi/8)
constexpr double kH = 0.70710678118654752440;   // sqrt(1/2)

// a * e^{-2 pi i m / 16}; m is a constant after unrolling, so the branches fold.
template <typename C>
__device__ __forceinline__ cx<C> rot16(cx<C> a, int m) {
    double c, s;
    switch (m & 15) {
        case 0: return a;
        case 4: return mkc<C>(a.y, -a.x);
        case 8: return mkc<C>(-a.x, -a.y);
        case 12: return mkc<C>(-a.y, a.x);
        case 1: c = kC1; s = kS1; break;
        case 2: c = kH; s = kH; break;
        case 3: c = kS1; s = kC1; break;
        case 5: c = -kS1; s = kC1; break;
        case 6: c = -kH; s = kH; break;
        case 7: c = -kC1; s = kS1; break;
        case 9: c = -kC1; s = -kS1; break;
        case 10: c = -kH; s = -kH; break;
        case 11: c = -kS1; s = -kC1; break;
        case 13: c = kS1; s = -kC1; break;
        case 14: c = kH; s = -kH; break;
        default: c = kC1; s = -kS1; break;
    }
    const C cc = (C)c, ss = (C)s;
    return mkc<C>(a.x * cc + a.y * ss, a.y * cc - a.x * ss);
}

__host__ __device__ constexpr int bit_rev(int q, int r) {
    int y = 0;
    for (int b = 1; b < r; b <<= 1) {
        y = (y << 1) | (q & 1);
        q >>= 1;
    }
    return y;
}

// r-point DFT in registers (r = 4, 8, 16): radix-2 decimation in frequency,
// result in bit-reversed order.
template <typename C, int r>
__device__ __forceinline__ void dft_small(cx<C> (&v)[r]) {
#pragma unroll
    for (int h = r / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int g = 0; g < r; g += 2 * h) {
#pragma unroll
            for (int j = 0; j < h; ++j) {
                const cx<C> a = v[g + j], b = v[g + j + h];
                v[g + j] = cadd(a, b);
                v[g + j + h] = rot16(csub(a, b), j * (16 / (2 * h)));
            }
        }
    }
}

// One Stockham pass of radix r (sub-transform length Ls before the pass) on
// the register layout x[s] = X[lane + 64 s]; the exchange goes through buf,
// the twiddles (tw[t] = e^{-2 pi i t / M}) are read through the caches.
template <typename C, int R, int r, int Ls>
__device__ __forceinline__ void fft_pass(cx<C> (&x)[R], cx<C>* buf, const cx<C>* __restrict__ tw, int lane) {
    constexpr int B = R / r;               // butterflies per lane
    constexpr int M = 64 * R;
    constexpr int span = M / (Ls * r);     // twiddle stride in tw
#pragma unroll
    for (int t = 0; t < B; ++t) {
        const int b = lane + 64 * t;
        const int j = b % Ls, k = b / Ls;
        cx<C> v[r];
#pragma unroll
        for (int i = 0; i < r; ++i) v[i] = x[t + i * B];
        if (Ls > 1) {
#pragma unroll
            for (int i = 1; i < r; ++i) v[i] = cmul(v[i], tw[j * i * span]);
        }
        dft_small<C, r>(v);
        const int base = k * Ls * r + j;
#pragma unroll
        for (int q = 0; q < r; ++q) buf[fpad(base + q * Ls)] = v[bit_rev(q, r)];
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < R; ++s) x[s] = buf[fpad(lane + 64 * s)];
    wave_sync();
}

template <typename C, int R>
__device__ __forceinline__ void fft_wave(cx<C> (&x)[R], cx<C>* buf, const cx<C>* __restrict__ tw, int lane) {
    if constexpr (R == 8) {
        fft_pass<C, 8, 8, 1>(x, buf, tw, lane);
        fft_pass<C, 8, 8, 8>(x, buf, tw, lane);
        fft_pass<C, 8, 8, 64>(x, buf, tw, lane);
    } else {
        static_assert(R == 16, "M = 512 or 1024");
        fft_pass<C, 16, 16, 1>(x, buf, tw, lane);
        fft_pass<C, 16, 16, 16>(x, buf, tw, lane);
        fft_pass<C, 16, 4, 256>(x, buf, tw, lane);
    }
}

// Bluestein: x[s] holds a[lane + 64 s] = u[j] c[j] (0 for j >= n); returns
// with x[s] = W[j] = DFT_n(u)[j] for j = lane + 64 s < n.  The table loads
// are issued one FFT ahead of their use.
template <typename C, int R>
__device__ __forceinline__ void bluestein(cx<C> (&x)[R], cx<C>* buf, const FftTables<C>& t, int lane) {
    cx<C> pre[R];
#pragma unroll
    for (int s = 0; s < R; ++s) pre[s] = t.bhat[lane + 64 * s];
    fft_wave<C, R>(x, buf, t.tw, lane);
#pragma unroll
    for (int s = 0; s < R; ++s) x[s] = cconj(cmul(x[s], pre[s]));
#pragma unroll
    for (int s = 0; s < R; ++s) pre[s] = t.chirp[lane + 64 * s];
    fft_wave<C, R>(x, buf, t.tw, lane);
    const C inv = (C)(1.0 / (64 * R));
#pragma unroll
    for (int s = 0; s < R; ++s) x[s] = cscale(cmul(cconj(x[s]), pre[s]), inv);
}

template <typename T, typename C, int R, int mode>
__global__ __launch_bounds__(256, (sizeof(C) == 4 || R == 8) ? 2 : 1) void k_tube_fft(TubeArgs a, FftTables<C> t) {
    using V = cx<C>;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ double s_red[2][4];
    const int n = a.n3;
    const int64_t N = a.N;
    T* tile = (T*)smem_raw;  // n rows of 16 tubes, pitch kFftLd
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    V* buf = (V*)(smem_raw + fft_tile_bytes(n, (int)sizeof(T))) + wave * fft_buf_entries(64 * R);
    const int64_t r0 = (int64_t)blockIdx.x * kFftTubes;
    double beta = 1.0;
    if (a.pX || a.eX) beta = a.beta_sched ? a.beta_sched[a.ctrl->iter] : a.beta_val;

    // load: element (tube q, position k) -> tile[k * kFftLd + q], 16-element runs
    int bad = 0;
    for (int e = tid; e < n * kFftTubes; e += 256) {
        const int k = e / kFftTubes, q = e - k * kFftTubes;
        const int64_t r = r0 + q;
        T v = (T)0;
        if (r < N) {
            const int64_t g = r + N * k;
            if (a.pX) v = (T)((double)((const T*)a.pX)[g] - (double)((const T*)a.pM)[g] / beta);
            else v = ((const T*)a.in)[g];
            if (a.check_finite && !isfinite((double)v)) bad = 1;
        }
        tile[k * kFftLd + q] = v;
    }
    if (a.check_finite && bad) atomicOr(&a.ctrl->status, kStNonFinite);
    __syncthreads();

    const C s0 = (C)sqrt(1.0 / n), s1 = (C)sqrt(2.0 / n);
    const int h = (n - 1) / 2;
    for (int pr = wave; pr < kFftTubes / 2; pr += 4) {
        const int q1 = 2 * pr, q2 = q1 + 1;
        if (r0 + q1 >= N) break;
        V x[R], cj[R], ph[R / 2];
        // table loads first, in one batch (the tables are zero-padded: no branches)
#pragma unroll
        for (int s = 0; s < R; ++s) cj[s] = t.chirp[lane + 64 * s];
        if constexpr (mode == kFftDctForward || mode == kFftDctInverse) {
#pragma unroll
            for (int s = 0; s < R / 2; ++s) ph[s] = t.phase[lane + 64 * s];
        }
        // chirped input a[j] = u[j] c[j]
#pragma unroll
        for (int s = 0; s < R; ++s) {
            const int j = lane + 64 * s;
            V u = mkc<C>((C)0, (C)0);
            if (j < n) {
                if constexpr (mode == kFftDctForward) {
                    const int src = (2 * j < n) ? 2 * j : 2 * (n - 1 - j) + 1;
                    u = mkc<C>((C)tile[src * kFftLd + q1], (C)tile[src * kFftLd + q2]);
                } else if constexpr (mode == kFftDftForward) {
                    u = mkc<C>((C)tile[j * kFftLd + q1], (C)tile[j * kFftLd + q2]);
                } else {
                    // U = V1 + i V2 from the coefficients; the input is conj(U)
                    V V1, V2;
                    if constexpr (mode == kFftDctInverse) {
                        const C sj = j == 0 ? s0 : s1;
                        const V w = cconj(ph[s < R / 2 ? s : 0]);  // j < n <= M/2: s < R/2
                        const C y1 = (C)tile[j * kFftLd + q1] / sj, y2 = (C)tile[j * kFftLd + q2] / sj;
                        const C z1 = j == 0 ? (C)0 : (C)tile[(n - j) * kFftLd + q1] / s1;
                        const C z2 = j == 0 ? (C)0 : (C)tile[(n - j) * kFftLd + q2] / s1;
                        V1 = cmul(w, mkc<C>(y1, -z1));
                        V2 = cmul(w, mkc<C>(y2, -z2));
                    } else {
                        int ir, ii;  // rows of Re and Im (-1: zero); isg: sign of Im
                        C isg = (C)1;
                        if (j == 0) { ir = 0; ii = -1; }
                        else if ((n & 1) == 0 && j == n / 2) { ir = n - 1; ii = -1; }
                        else if (j <= h) { ir = 2 * j - 1; ii = 2 * j; }
                        else { ir = 2 * (n - j) - 1; ii = 2 * (n - j); isg = (C)-1; }
                        V1 = mkc<C>((C)tile[ir * kFftLd + q1],
                                          ii < 0 ? (C)0 : isg * (C)tile[ii * kFftLd + q1]);
                        V2 = mkc<C>((C)tile[ir * kFftLd + q2],
                                          ii < 0 ? (C)0 : isg * (C)tile[ii * kFftLd + q2]);
                    }
                    u = mkc<C>(V1.x - V2.y, -(V1.y + V2.x));
                }
            }
            x[s] = cmul(u, cj[s]);
        }
        bluestein<C, R>(x, buf, t, lane);
        if constexpr (mode == kFftDctForward || mode == kFftDftForward) {
            // separate the two tubes' spectra: needs W[n - k], from the exchange buffer
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int j = lane + 64 * s;
                if (j < n) buf[fpad(j)] = x[s];
            }
            wave_sync();
#pragma unroll
            for (int s = 0; s < R / 2; ++s) {
                const int k = lane + 64 * s;
                if (k >= n) break;
                if constexpr (mode == kFftDctForward) {
                    const V Wk = buf[fpad(k)], Wn = cconj(buf[fpad(k == 0 ? 0 : n - k)]);
                    const V V1 = cscale(cadd(Wk, Wn), (C)0.5);
                    const V d = csub(Wk, Wn);
                    const V V2 = mkc<C>((C)0.5 * d.y, (C)-0.5 * d.x);
                    const V p = ph[s];
                    const C sk = k == 0 ? s0 : s1;
                    tile[k * kFftLd + q1] = (T)(sk * (p.x * V1.x - p.y * V1.y));
                    tile[k * kFftLd + q2] = (T)(sk * (p.x * V2.x - p.y * V2.y));
                } else {
                    int f, im;
                    if (k == 0) { f = 0; im = 0; }
                    else if ((n & 1) == 0 && k == n - 1) { f = n / 2; im = 0; }
                    else { f = (k + 1) / 2; im = (k & 1) ? 0 : 1; }
                    const V Wk = buf[fpad(f)], Wn = cconj(buf[fpad(f == 0 ? 0 : n - f)]);
                    const V V1 = cscale(cadd(Wk, Wn), (C)0.5);
                    const V d = csub(Wk, Wn);
                    const V V2 = mkc<C>((C)0.5 * d.y, (C)-0.5 * d.x);
                    tile[k * kFftLd + q1] = (T)(im ? V1.y : V1.x);
                    tile[k * kFftLd + q2] = (T)(im ? V2.y : V2.x);
                }
            }
            wave_sync();
        } else {
            // v1 + i v2 = conj(W) / n
            const C invn = (C)(1.0 / n);
#pragma unroll
            for (int s = 0; s < R; ++s) {
                const int j = lane + 64 * s;
                if (j < n) {
                    const int dst = (mode == kFftDftInverse) ? j : ((2 * j < n) ? 2 * j : 2 * (n - 1 - j) + 1);
                    tile[dst * kFftLd + q1] = (T)(x[s].x * invn);
                    tile[dst * kFftLd + q2] = (T)(-x[s].y * invn);
                }
            }
            wave_sync();
        }
    }
    __syncthreads();

    // store (and the completion epilogue), 16-element runs
    double dn = 0.0, xn = 0.0;
    for (int e = tid; e < n * kFftTubes; e += 256) {
        const int k = e / kFftTubes, q = e - k * kFftTubes;
        const int64_t r = r0 + q;
        if (r >= N) continue;
        const int64_t g = r + N * k;
        const T y = tile[k * kFftLd + q];
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
    int M = 512;
    while (M < 2 * n - 1) M <<= 1;
    return M;
}

// prec: 0 FP64 tables (double data), else FP32 tables (float data).
size_t fft_table_bytes(int n, int prec) {
    const int M = fft_size(n);
    return (prec == 0 ? sizeof(double) : sizeof(float)) * 2 * ((size_t)M + M + M + M / 2);
}

template <typename C>
static void write_tables(int n, C* out) {
    const int M = fft_size(n);
    const long double pi = acosl(-1.0L);
    C* tw = out;          // M complex
    C* ch = tw + 2 * M;   // M complex (n values, then zeros)
    C* bh = ch + 2 * M;   // M complex
    C* ph = bh + 2 * M;   // M/2 complex (n values, then zeros)
    for (int j = 2 * n; j < 2 * M; ++j) ch[j] = (C)0;
    for (int j = 2 * n; j < M; ++j) ph[j] = (C)0;
    std::vector<std::complex<long double>> root(M), c(n), b(M, 0.0L);
    for (int j = 0; j < M; ++j) {
        const long double ang = -2.0L * pi * j / M;
        root[j] = std::complex<long double>(cosl(ang), sinl(ang));
        tw[2 * j] = (C)root[j].real();
        tw[2 * j + 1] = (C)root[j].imag();
    }
    for (int j = 0; j < n; ++j) {
        const long long q = ((long long)j * j) % (2LL * n);
        const long double ang = -pi * (long double)q / n;
        c[j] = std::complex<long double>(cosl(ang), sinl(ang));
        ch[2 * j] = (C)c[j].real();
        ch[2 * j + 1] = (C)c[j].imag();
    }
    // wrapped conj(c): b[m] = conj(c[m]) for m < n, b[M - m] = conj(c[m]) for 0 < m < n
    for (int m = 0; m < n; ++m) {
        b[m] = std::conj(c[m]);
        if (m > 0) b[M - m] = std::conj(c[m]);
    }
    for (int k = 0; k < M; ++k) {
        std::complex<long double> acc = 0.0L;
        for (int m = 0; m < M; ++m) {
            if (m >= n && m <= M - n) continue;  // zero entries
            acc += b[m] * root[((long long)k * m) % M];
        }
        bh[2 * k] = (C)acc.real();
        bh[2 * k + 1] = (C)acc.imag();
    }
    for (int k = 0; k < n; ++k) {
        const long double ang = -pi * k / (2.0L * n);
        ph[2 * k] = (C)cosl(ang);
        ph[2 * k + 1] = (C)sinl(ang);
    }
}

// Tables (computed in long double, stored in FP64 or FP32): twiddles
// e^{-2 pi i t/M}; chirp c[j] = e^{-i pi (j^2 mod 2n)/n} (zero-padded to M);
// the FFT of the wrapped conjugate chirp (a direct O(M^2) DFT over the
// twiddles, once per length); DCT phases e^{-i pi k/(2n)} (zero-padded to M/2).
void make_fft_tables(int n, int prec, void* out) {
    if (prec == 0) write_tables<double>(n, (double*)out);
    else write_tables<float>(n, (float*)out);
}

int fft_lds_bytes(int n, int prec) {
    const int es = prec == 0 ? 8 : 4;
    return fft_tile_bytes(n, es) + 4 * fft_buf_entries(fft_size(n)) * 2 * es;
}

bool fft_fits(int n3) { return n3 > kMaxTube && fft_size(n3) <= 1024 && fft_lds_bytes(n3, 0) <= kLdsBudget; }

template <typename T, typename C, int R, int mode>
static hipError_t launch_fft(const TubeArgs& a, const FftTables<C>& t, int lds, dim3 grid, hipStream_t s) {
    hipError_t e = hipFuncSetAttribute((const void*)k_tube_fft<T, C, R, mode>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tube_fft<T, C, R, mode>), grid, dim3(256), lds, s, a, t);
    return hipGetLastError();
}

template <typename T, typename C, int R>
static hipError_t launch_fft_mode(const TubeArgs& a, const FftTables<C>& t, int mode, int lds, dim3 grid,
                                  hipStream_t s) {
    switch (mode) {
        case kFftDctForward: return launch_fft<T, C, R, kFftDctForward>(a, t, lds, grid, s);
        case kFftDctInverse: return launch_fft<T, C, R, kFftDctInverse>(a, t, lds, grid, s);
        case kFftDftForward: return launch_fft<T, C, R, kFftDftForward>(a, t, lds, grid, s);
        case kFftDftInverse: return launch_fft<T, C, R, kFftDftInverse>(a, t, lds, grid, s);
        default: return hipErrorInvalidValue;
    }
}

template <typename T, typename C>
static hipError_t launch_fft_typed(const TubeArgs& a, const void* tables, int mode, hipStream_t s) {
    const int n = a.n3, M = fft_size(n);
    FftTables<C> t;
    const cx<C>* p = (const cx<C>*)tables;
    t.tw = p;
    t.chirp = p + M;
    t.bhat = p + 2 * M;
    t.phase = p + 3 * M;
    t.n = n;
    const int lds = fft_lds_bytes(n, sizeof(C) == 8 ? 0 : 1);
    const dim3 grid((unsigned)((a.N + kFftTubes - 1) / kFftTubes));
    return M == 512 ? launch_fft_mode<T, C, 8>(a, t, mode, lds, grid, s)
                    : launch_fft_mode<T, C, 16>(a, t, mode, lds, grid, s);
}

hipError_t launch_tube_fft(int prec, const TubeArgs& a, const void* tables, int mode, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    if (!fft_fits(a.n3)) return hipErrorInvalidValue;
    return prec == 0 ? launch_fft_typed<double, double>(a, tables, mode, s)
                     : launch_fft_typed<float, float>(a, tables, mode, s);
}

}  // namespace tsvd
