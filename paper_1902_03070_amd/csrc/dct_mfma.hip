// Tube transforms on the matrix cores.
//
// Xbar = dct(X,[],3) (Section 3) is, on the mode-3 unfolding, a dense
// contraction over the tube index:  out[k'][r] = sum_k M[k'][k] in[r + N k]
// with M = C (forward) or C^T (inverse).  Each wavefront takes 32 consecutive
// tubes (two 16-wide column blocks), loads their whole tubes once (the
// completion prologue Z = X - Mlt/beta is applied on the fly), and for every
// 16-row block of M accumulates the product with MFMA instructions:
//   engine 0 (FP64):  v_mfma_f64_16x16x4f64
//   engine 1 (FP32):  v_mfma_f32_16x16x4f32
//   engine 2 (BF16 hi+lo, FP32 data): v_mfma_f32_16x16x32_bf16 three times,
//       M_hi x_hi + M_hi x_lo + M_lo x_hi, with v = v_hi + v_lo the split of a
//       float into two bfloat16 values (the lo*lo term is dropped).
// M arrives pre-arranged in fragment order (see make_tube_fragments), so every
// A-operand load is one contiguous 64-lane read.  Results are written per
// output row as 16-tube runs; the completion epilogue (Algorithm 1 X- and
// M-updates and the norms of the relative change) is applied per element.
//
// Lane layouts (gfx950): A 16xK operand, lane l holds rows l%16 and K slice
// l/16; B Kx16 operand, lane l holds column l%16 and K slice l/16; result:
// FP64 element v of lane l is row l/16 + 4v, FP32 element v is row 4(l/16)+v,
// column l%16 in both.
#include <string.h>

#include "internal.h"

namespace tsvd {

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int kTubeBlocks = 2;  // 16-tube column blocks per wavefront

template <int ENG> struct Eng;
template <> struct Eng<0> { typedef double T; typedef double A; typedef d4_t Acc; static constexpr int KSTEP = 4; };
template <> struct Eng<1> { typedef float T; typedef float A; typedef f4_t Acc; static constexpr int KSTEP = 4; };
template <> struct Eng<2> { typedef float T; typedef bf8_t A; typedef f4_t Acc; static constexpr int KSTEP = 32; };

template <int ENG>
__device__ __forceinline__ int out_row(int lane, int v) {
    return ENG == 0 ? (lane >> 4) + 4 * v : 4 * (lane >> 4) + v;
}

template <typename T>
__device__ __forceinline__ T load_in(const TubeArgs& a, int64_t e, double beta) {
    if (a.pX) return (T)((double)((const T*)a.pX)[e] - (double)((const T*)a.pM)[e] / beta);
    return ((const T*)a.in)[e];
}

template <int ENG, int KS>
__global__ __launch_bounds__(256) void k_tube_mfma(TubeArgs a, const void* __restrict__ frag) {
    typedef typename Eng<ENG>::T T;
    typedef typename Eng<ENG>::Acc Acc;
    constexpr int KSTEP = Eng<ENG>::KSTEP;
    constexpr int KE = (ENG == 2) ? 8 : 1;  // B values per lane per K step
    __shared__ double s_red[2][4];
    const int n3 = a.n3;
    const int64_t N = a.N;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int col = lane & 15, kq = lane >> 4;
    const int MB = (n3 + 15) >> 4;
    double beta = 1.0;
    if (a.pX || a.eX) beta = a.beta_sched ? a.beta_sched[a.ctrl->iter] : a.beta_val;
    double dn = 0.0, xn = 0.0;
    int bad = 0;
#pragma unroll 1
    for (int tb = 0; tb < kTubeBlocks; ++tb) {
        const int64_t r0 = (((int64_t)blockIdx.x * 4 + wave) * kTubeBlocks + tb) * 16;
        if (r0 >= N) break;
        const int64_t r = r0 + col;
        const bool live = r < N;
        // the lane's slice of the whole tube: KS steps x KE values
        T xv[KS * KE];
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int e = 0; e < KE; ++e) {
                const int k = ks * KSTEP + kq * KE + e;
                T v = (T)0;
                if (live && k < n3) {
                    v = load_in<T>(a, r + N * k, beta);
                    if (a.check_finite && !isfinite((double)v)) bad = 1;
                }
                xv[ks * KE + e] = v;
            }
        // BF16 engine: split every value into hi + lo bfloat16 parts
        bf8_t bh[ENG == 2 ? KS : 1], bl[ENG == 2 ? KS : 1];
        if constexpr (ENG == 2) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks)
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float x = (float)xv[ks * 8 + e];
                    const __bf16 hb = (__bf16)x;
                    bh[ks][e] = hb;
                    bl[ks][e] = (__bf16)(x - (float)hb);
                }
        }
#pragma unroll 1
        for (int mb = 0; mb < MB; ++mb) {
            Acc acc;
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[v] = 0;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int64_t fi = ((int64_t)mb * KS + ks) * 64 + lane;
                if constexpr (ENG == 0) {
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(((const double*)frag)[fi], (double)xv[ks], acc, 0, 0, 0);
                } else if constexpr (ENG == 1) {
                    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(((const float*)frag)[fi], (float)xv[ks], acc, 0, 0, 0);
                } else {
                    const int64_t nfr = (int64_t)MB * KS * 64;
                    const bf8_t ah = ((const bf8_t*)frag)[fi];
                    const bf8_t al = ((const bf8_t*)frag)[nfr + fi];
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[ks], acc, 0, 0, 0);
                    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh[ks], acc, 0, 0, 0);
                }
            }
            if (!live) continue;
            if (!a.eX) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int ko = mb * 16 + out_row<ENG>(lane, v);
                    if (a.out && ko < n3) ((T*)a.out)[r + N * ko] = (T)acc[v];
                }
                continue;
            }
            // completion epilogue: every input of the block's four rows is loaded before
            // the first store (one memory round trip per block; B is read whether or not
            // the entry is observed, so no load waits on the mask)
            T* X = (T*)a.eX;
            T* Ml = (T*)a.eM;
            T xo[4], mo[4], bo[4];
            unsigned char mk[4];
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ko = mb * 16 + out_row<ENG>(lane, v);
                xo[v] = mo[v] = bo[v] = (T)0;
                mk[v] = 0;
                if (ko < n3) {
                    const int64_t e = r + N * ko;
                    xo[v] = X[e];
                    mo[v] = Ml[e];
                    bo[v] = ((const T*)a.eB)[e];
                    mk[v] = a.emask[e];
                }
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int ko = mb * 16 + out_row<ENG>(lane, v);
                if (ko >= n3) continue;
                const int64_t e = r + N * ko;
                const T y = (T)acc[v];
                if (a.out) ((T*)a.out)[e] = y;
                const T xold = xo[v];
                const T mold = mo[v];
                const T xnew = mk[v] ? bo[v] : (T)((double)y + (double)mold / beta);
                Ml[e] = (T)((double)mold + beta * ((double)y - (double)xnew));
                X[e] = xnew;
                const double d = (double)xnew - (double)xold;
                dn += d * d;
                xn += (double)xold * (double)xold;
            }
        }
    }
    if (a.check_finite && bad) atomicOr(&a.ctrl->status, kStNonFinite);
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
        if (threadIdx.x == 0) {
            // kNormSlots slot pairs spread the atomics of the workgroups over addresses
            double* slot = a.norms + 2 * (blockIdx.x % kNormSlots);
            atomicAdd(slot, s_red[0][0] + s_red[0][1] + s_red[0][2] + s_red[0][3]);
            atomicAdd(slot + 1, s_red[1][0] + s_red[1][1] + s_red[1][2] + s_red[1][3]);
        }
    }
}

// Fragment-ordered copy of the row-major n3 x n3 matrix M (FP64 on the host).
// Engines 0/1: element [(mb*KS + ks)*64 + lane] = M[mb*16 + lane%16][ks*4 + lane/16].
// Engine 2: two bf16 arrays (hi, then lo), 8 values per lane:
//   [((mb*KS + ks)*64 + lane)*8 + e] = split(M[mb*16 + lane%16][ks*32 + 8*(lane/16) + e]).
// Out-of-range entries are zero.  Returns the byte size written to *out.
static uint16_t bf16_bits_rne(float x) {
    uint32_t u;
    memcpy(&u, &x, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}
static float bf16_to_float(uint16_t b) {
    const uint32_t u = (uint32_t)b << 16;
    float f;
    memcpy(&f, &u, 4);
    return f;
}

// K steps the kernel is instantiated for (the fragment array uses the same
// padded count): engine 2 exact (1..4), engines 0/1 rounded up to 2,4,8,16,24,32.
int tube_ks(int eng, int n3) {
    if (eng == 2) return (n3 + 31) / 32;
    const int ks = (n3 + 3) / 4;
    if (ks <= 2) return 2;
    if (ks <= 4) return 4;
    if (ks <= 8) return 8;
    if (ks <= 16) return 16;
    if (ks <= 24) return 24;
    return 32;
}

size_t tube_fragment_bytes(int eng, int n3) {
    const size_t n = (size_t)((n3 + 15) / 16) * tube_ks(eng, n3) * 64;
    return eng == 0 ? n * 8 : eng == 1 ? n * 4 : n * 8 * 2 * 2;
}

void make_tube_fragments(int eng, int n3, const double* M, void* out) {
    const int KS = tube_ks(eng, n3), MB = (n3 + 15) / 16;
    const size_t nfr = (size_t)MB * KS * 64;
    for (int mb = 0; mb < MB; ++mb)
        for (int ks = 0; ks < KS; ++ks)
            for (int lane = 0; lane < 64; ++lane) {
                const size_t fi = ((size_t)mb * KS + ks) * 64 + lane;
                const int row = mb * 16 + lane % 16;
                if (eng != 2) {
                    const int k = ks * 4 + lane / 16;
                    const double v = (row < n3 && k < n3) ? M[(size_t)row * n3 + k] : 0.0;
                    if (eng == 0) ((double*)out)[fi] = v;
                    else ((float*)out)[fi] = (float)v;
                } else {
                    for (int e = 0; e < 8; ++e) {
                        const int k = ks * 32 + 8 * (lane / 16) + e;
                        const float v = (row < n3 && k < n3) ? (float)M[(size_t)row * n3 + k] : 0.0f;
                        const uint16_t hi = bf16_bits_rne(v);
                        const uint16_t lo = bf16_bits_rne(v - bf16_to_float(hi));
                        ((uint16_t*)out)[fi * 8 + e] = hi;
                        ((uint16_t*)out)[(nfr + fi) * 8 + e] = lo;
                    }
                }
            }
}

template <int ENG, int KS>
static void launch_ks(const TubeArgs& a, const void* frag, hipStream_t s) {
    const int64_t per_wg = 4 * kTubeBlocks * 16;
    dim3 grid((unsigned)((a.N + per_wg - 1) / per_wg)), block(256);
    hipLaunchKernelGGL((k_tube_mfma<ENG, KS>), grid, block, 0, s, a, frag);
}

template <int ENG>
static hipError_t launch_eng(const TubeArgs& a, const void* frag, hipStream_t s) {
    const int ks = tube_ks(ENG, a.n3);
    if constexpr (ENG == 2) {
        switch (ks) {
            case 1: launch_ks<ENG, 1>(a, frag, s); break;
            case 2: launch_ks<ENG, 2>(a, frag, s); break;
            case 3: launch_ks<ENG, 3>(a, frag, s); break;
            case 4: launch_ks<ENG, 4>(a, frag, s); break;
            default: return hipErrorInvalidValue;
        }
    } else {
        switch (ks) {
            case 2: launch_ks<ENG, 2>(a, frag, s); break;
            case 4: launch_ks<ENG, 4>(a, frag, s); break;
            case 8: launch_ks<ENG, 8>(a, frag, s); break;
            case 16: launch_ks<ENG, 16>(a, frag, s); break;
            case 24: launch_ks<ENG, 24>(a, frag, s); break;
            case 32: launch_ks<ENG, 32>(a, frag, s); break;
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

// The transform matrix built on the device, for callers that keep it in
// memory the library did not allocate.  Entry (row, col) of M is C[row][col]
// forward and C[col][row] inverse, with the orthonormal DCT-II
// C[k][t] = s_k cos(pi (2t + 1) k / (2 n3)), s_0 = sqrt(1/n3), s_k = sqrt(2/n3)
// (Section 3, dct(., [], 3)), evaluated in FP64 with the same expression as
// the host copy.  dense = 1: row-major n3 x n3 in FP64 (eng 0) or FP32
// (otherwise), the vector-ALU kernel's operand; dense = 0: the fragment order
// of make_tube_fragments for engine eng, KS = tube_ks(eng, n3).
__device__ __forceinline__ double dct_entry(int n3, int k, int t) {
    const double sk = k == 0 ? sqrt(1.0 / n3) : sqrt(2.0 / n3);
    return sk * cos(3.141592653589793 * (2.0 * t + 1.0) * k / (2.0 * n3));
}

__device__ __forceinline__ unsigned short bf16_rne_dev(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__global__ void k_tube_matrix(int eng, int n3, int inverse, int KS, int dense, void* out, int64_t total) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    if (dense) {
        const int row = (int)(idx / n3), col = (int)(idx % n3);
        const double v = inverse ? dct_entry(n3, col, row) : dct_entry(n3, row, col);
        if (eng == 0) ((double*)out)[idx] = v;
        else ((float*)out)[idx] = (float)v;
        return;
    }
    const int64_t nfr = (int64_t)((n3 + 15) / 16) * KS * 64;
    if (eng != 2) {
        const int lane = (int)(idx % 64), ks = (int)((idx / 64) % KS), mb = (int)(idx / 64 / KS);
        const int row = mb * 16 + lane % 16, k = ks * 4 + lane / 16;
        double v = 0.0;
        if (row < n3 && k < n3) v = inverse ? dct_entry(n3, k, row) : dct_entry(n3, row, k);
        if (eng == 0) ((double*)out)[idx] = v;
        else ((float*)out)[idx] = (float)v;
        return;
    }
    const int e = (int)(idx % 8);
    const int64_t fi = idx / 8;
    const int lane = (int)(fi % 64), ks = (int)((fi / 64) % KS), mb = (int)(fi / 64 / KS);
    const int row = mb * 16 + lane % 16, k = ks * 32 + 8 * (lane / 16) + e;
    float v = 0.0f;
    if (row < n3 && k < n3) v = (float)(inverse ? dct_entry(n3, k, row) : dct_entry(n3, row, k));
    const unsigned short hi = bf16_rne_dev(v);
    const unsigned short lo = bf16_rne_dev(v - __uint_as_float((uint32_t)hi << 16));
    ((unsigned short*)out)[fi * 8 + e] = hi;
    ((unsigned short*)out)[(nfr + fi) * 8 + e] = lo;
}

size_t tube_matrix_bytes(int eng, int n3) {
    if (n3 <= kMaxTube) return tube_fragment_bytes(eng, n3);
    return (size_t)n3 * n3 * (eng == 0 ? 8 : 4);
}

hipError_t launch_tube_matrix(int eng, int n3, int inverse, void* out, hipStream_t s) {
    if (n3 <= 0) return hipErrorInvalidValue;
    const int dense = n3 > kMaxTube ? 1 : 0;
    const int KS = dense ? 0 : tube_ks(eng, n3);
    int64_t total;
    if (dense) total = (int64_t)n3 * n3;
    else total = (int64_t)((n3 + 15) / 16) * KS * 64 * (eng == 2 ? 8 : 1);
    const int threads = 256;
    hipLaunchKernelGGL(k_tube_matrix, dim3((unsigned)((total + threads - 1) / threads)), dim3(threads), 0, s, eng,
                       n3, inverse, KS, dense, out, total);
    return hipGetLastError();
}

hipError_t launch_tube_mfma(int eng, const TubeArgs& a, const void* frag, hipStream_t s) {
    if (a.N <= 0) return hipSuccess;
    if (a.n3 > kMaxTube) return hipErrorInvalidValue;
    if (eng == 0) return launch_eng<0>(a, frag, s);
    if (eng == 1) return launch_eng<1>(a, frag, s);
    return launch_eng<2>(a, frag, s);
}

}  // namespace tsvd
