// Batched one-sided (Hestenes) Jacobi SVD of the transformed frontal slices.
//
// The method takes the SVD of every frontal slice of Zbar = dct(Z,[],3)
// (Theorem 4; Algorithm 1, per-slice SVD).  Each slice is handled in "tall"
// form T (m x p, m >= p): the slice itself, or its transpose when n1 < n2.
// Columns of T are rotated in pairs until every pair is orthogonal to a
// tolerance tol (m u for FP64, u = 2^-53; 2 sqrt(m) u32 for FP32 sweeps, since
// FP32 rounding of the stored columns bounds the attainable orthogonality;
// m u32 for the FP32 sweeps of the mixed path, which ends with one sweep at
// m u whose inner products and angles are FP64):
//     alpha = |x|^2, beta = |y|^2 (FP64 sums), gamma = x.y (FP64 sums; FP32
//     for FP32 sweeps of the team kernel)
//     rotate iff gamma^2 > tol^2 alpha beta
//     zeta = (beta - alpha) / (2 gamma),  t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2))
//     c = 1 / sqrt(1 + t^2),  s = c t,  x' = c x - s y,  y' = s x + c y.
// On exit A holds T V (columns = sigma_j u_j); V is accumulated only when asked.
//
// Work decomposition.  A column pair is handled by a group of G lanes (G = 16
// or 32, chosen by the tuner; 64 in the team kernel), each lane holding R rows
// (rows l, l+G, ..., so LDS accesses of a group are contiguous).  The dot
// products are reduced inside the group with DPP row operations (plus one or
// two lane swaps for G = 32, 64); a wavefront therefore works on 64/G pairs
// at once.
//
//  * resident kernel: one workgroup per slice, the whole slice (and V) in LDS,
//    circle-method round robin over all columns (p/2 disjoint pairs per round).
//  * team kernel: slices too large for LDS.  Columns are cut into nb blocks of
//    b; a round-robin tournament over blocks gives nb/2 disjoint block pairs
//    per step.  Each of the W workgroups of a team holds one block pair: the J
//    block in LDS and, during the b cross rounds, each I column in the
//    registers of its own lane group (only J columns move through LDS).  The
//    first step of a sweep also orthogonalizes the pairs inside each block.
//    Blocks go back to global memory (the XCD's L2) after each step; within a
//    sweep each block passes from its holder to the next one through a flag,
//    and the sweep ends at a team barrier.  The grid is sized so that every
//    workgroup of a team is resident (ordinary launches by default, cooperative
//    ones on request outside graph capture); every wait is bounded and reports
//    a timeout instead of hanging.
#include <algorithm>

#include "jacobi.h"

namespace tsvd {

template <typename T> struct Unit;
template <> struct Unit<double> { static constexpr double v = 1.1102230246251565e-16; };  // 2^-53
template <> struct Unit<float> { static constexpr double v = 5.9604644775390625e-08; };    // 2^-24

// DPP move of a double (two 32-bit halves).  CTRL: 0xB1 = quad_perm [1,0,3,2],
// 0x4E = quad_perm [2,3,0,1], 0x141 = row_half_mirror, 0x140 = row_mirror.
// These patterns read a valid lane for every lane, so the old value is never
// used (passing the source keeps the compiler from materialising one).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int l = __double2loint(v), h = __double2hiint(v);
    const int lo = __builtin_amdgcn_update_dpp(l, l, CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(h, h, CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Sum of the two 16-lane rows of each 32-lane half: v_permlane16_swap of a
// value with itself leaves row 2r in one result and row 2r+1 in the other, in
// both rows, so every lane adds the same two values in the same order.
__device__ __forceinline__ double pair_rows_sum(double v) {
    const unsigned l = (unsigned)__double2loint(v), h = (unsigned)__double2hiint(v);
    const auto a = __builtin_amdgcn_permlane16_swap(l, l, false, false);
    const auto b = __builtin_amdgcn_permlane16_swap(h, h, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// Sum of the two 32-lane halves of the wavefront: v_permlane32_swap of a value
// with itself leaves the lower half's value in one result and the upper
// half's in the other, in every lane, so every lane adds them in one order.
__device__ __forceinline__ double halves_sum(double v) {
    const unsigned l = (unsigned)__double2loint(v), h = (unsigned)__double2hiint(v);
    const auto a = __builtin_amdgcn_permlane32_swap(l, l, false, false);
    const auto b = __builtin_amdgcn_permlane32_swap(h, h, false, false);
    return __hiloint2double((int)b[0], (int)a[0]) + __hiloint2double((int)b[1], (int)a[1]);
}

// Sum over a group of G lanes (G = 16: one DPP row; G = 32: two rows; G = 64:
// the wavefront).  Each step adds a value to its mirror image, so every lane
// of the group ends with the same bits.
template <int G>
__device__ __forceinline__ double group_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    v += dpp_d<0x140>(v);
    if (G >= 32) v = pair_rows_sum(v);
    if (G == 64) v = halves_sum(v);
    return v;
}

// The same sum for an FP32 value: one DPP add per step instead of two moves
// and an FP64 add.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    const int i = __float_as_int(v);
    return __int_as_float(__builtin_amdgcn_update_dpp(i, i, CTRL, 0xF, 0xF, true));
}
template <int G>
__device__ __forceinline__ float group_sum_f(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    if (G >= 32) {
        const unsigned u = __float_as_uint(v);
        const auto a = __builtin_amdgcn_permlane16_swap(u, u, false, false);
        v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    }
    if (G == 64) {
        const unsigned u = __float_as_uint(v);
        const auto a = __builtin_amdgcn_permlane32_swap(u, u, false, false);
        v = __uint_as_float(a[0]) + __uint_as_float(a[1]);
    }
    return v;
}

// Circle-method round robin on n (even) players: round s (0..n-2), pair q
// (0..n/2-1) -> players (i < j).  Every pair meets exactly once in n-1 rounds.
// (s + q and s - q stay within one period of n - 1, so a conditional add or
// subtract replaces the remainder.)
__device__ __forceinline__ void rr_pair(int s, int q, int n, int& i, int& j) {
    int a, b;
    if (q == 0) {
        a = n - 1;
        b = s;
    } else {
        a = s + q;
        if (a >= n - 1) a -= n - 1;
        b = s - q;
        if (b < 0) b += n - 1;
    }
    i = a < b ? a : b;
    j = a < b ? b : a;
}

// Load of a value another workgroup of the team stored: a device-scope
// relaxed load (sc1), which misses the CU's L1 and reads the XCD's L2, where
// the partner's acknowledged stores are.  This replaces an acquire fence (an
// L1 and L2 invalidation) at every team barrier.
template <typename T>
__device__ __forceinline__ T ld_team(const T* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Reciprocal and reciprocal square root: hardware estimate plus one Newton
// step (close to full FP64 precision).
__device__ __forceinline__ double rcp_nr(double x) {
    double r = __builtin_amdgcn_rcp(x);
    return r * fma(-x, r, 2.0);
}
__device__ __forceinline__ double rsq_nr(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    return y * fma(-0.5 * x * y, y, 1.5);
}

// Rotation parameters from the column norms a = |x|^2, b = |y|^2 and the
// group-reduced g = x.y.  Returns false when the pair is already orthogonal
// to tol.  With d = b - a the tangent
//     t = sgn(zeta) / (|zeta| + sqrt(1 + zeta^2)),  zeta = d / (2 g),
// is evaluated as t = sgn(zeta) |2g| / den, den = |d| + r, r = sqrt(d^2 + 4 g^2)
// (multiply through by |2g|; sgn(0) = +1).  Since 1 + t^2 = 2 r / den, c and s
// both follow from one reciprocal square root z = 1/sqrt(2 r den): c = den z,
// s = sgn |2g| z, and t = s / c = sgn |2g| 2 r z^2.  Two reciprocal square
// roots and no reciprocal; c^2 + s^2 = 1 to working precision, so the rotation
// is orthogonal.  After it, |x'|^2 = a - t g and |y'|^2 = b + t g.
__device__ __forceinline__ bool needs_rotation(double a, double b, double g, double tol) {
    return !(g == 0.0 || g * g <= (tol * tol) * (a * b));
}
__device__ __forceinline__ void rotation_angle(double a, double b, double g, double& c, double& s, double& t) {
    const double d = b - a;
    const double w = fma(d, d, 4.0 * (g * g));  // r^2, r = sqrt(d^2 + 4 g^2)
    const double r = w * rsq_nr(w);
    const double den = fabs(d) + r;              // t = sgn 2|g| / den
    // 1 + t^2 = 2 r / den, so with z = 1/sqrt(2 r den):  c = den z,  |s| = 2|g| z,
    // and 1/den = 2 r z^2 gives t without a reciprocal
    const double z = rsq_nr(2.0 * r * den);
    const double ag2 = 2.0 * fabs(g);
    // sgn(zeta) = + exactly when d g >= 0 (d = 0 gives +0 or -0, both >= 0): a select, no branch
    const double sg = d * g >= 0.0 ? ag2 : -ag2;
    c = den * z;
    s = sg * z;
    t = sg * (2.0 * r * z * z);
}
__device__ __forceinline__ bool rotation(double a, double b, double g, double tol, double& c, double& s,
                                         double& t) {
    if (!needs_rotation(a, b, g, tol)) return false;
    rotation_angle(a, b, g, c, s, t);
    return true;
}

// Partial inner product of a lane's R rows of x and y (and, when norms is
// set, the partial squared norms).  FP32 data accumulate their R products in
// FP32 unless f64 (refinement sweep) asks for FP64.
template <typename T, int R>
__device__ __forceinline__ double partial_dot(const T* x, const T* y, bool f64) {
    // four independent accumulators shorten the dependency chain
    if (sizeof(T) == 8 || f64) {
        double p0 = 0.0, p1 = 0.0, p2 = 0.0, p3 = 0.0;
#pragma unroll
        for (int q = 0; q < R; q += 4) {
            p0 = fma((double)x[q], (double)y[q], p0);
            p1 = fma((double)x[q + 1], (double)y[q + 1], p1);
            p2 = fma((double)x[q + 2], (double)y[q + 2], p2);
            p3 = fma((double)x[q + 3], (double)y[q + 3], p3);
        }
        return (p0 + p1) + (p2 + p3);
    }
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
    for (int q = 0; q < R; q += 4) {
        p0 = fmaf((float)x[q], (float)y[q], p0);
        p1 = fmaf((float)x[q + 1], (float)y[q + 1], p1);
        p2 = fmaf((float)x[q + 2], (float)y[q + 2], p2);
        p3 = fmaf((float)x[q + 3], (float)y[q + 3], p3);
    }
    return (double)((p0 + p1) + (p2 + p3));
}

// Group-reduced inner product of the first R values of x and y.  FP32 data
// outside an FP64 sweep are summed in FP32 throughout (lane partials and the
// reduction): the error, a few units of 2^-24 times |x||y|, stays far below
// every rotation threshold used with FP32 data.
template <typename T, int R, int G>
__device__ __forceinline__ double group_dot(const T* x, const T* y, bool f64) {
    if (sizeof(T) == 4 && !f64) {
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
        for (int q = 0; q < R; q += 4) {
            p0 = fmaf((float)x[q], (float)y[q], p0);
            p1 = fmaf((float)x[q + 1], (float)y[q + 1], p1);
            p2 = fmaf((float)x[q + 2], (float)y[q + 2], p2);
            p3 = fmaf((float)x[q + 3], (float)y[q + 3], p3);
        }
        return (double)group_sum_f<G>((p0 + p1) + (p2 + p3));
    }
    return group_sum<G>(partial_dot<T, R>(x, y, f64));
}

template <typename T, int R>
__device__ __forceinline__ double partial_norm(const T* x) {
    double pa = 0.0;
#pragma unroll
    for (int q = 0; q < R; ++q) pa = fma((double)x[q], (double)x[q], pa);
    return pa;
}

// Rotations run in the data's precision: the cosine and sine are rounded to
// T once and each rotated value takes a product and an FMA.  In the mixed
// path's FP64 sweep the inner products and angles are FP64 while the
// rotation arithmetic stays FP32, the precision the values are stored in.
template <typename T, int R>
__device__ __forceinline__ void rotate_regs(T (&x)[R], T (&y)[R], double c, double s) {
    const T cc = (T)c, ss = (T)s;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const T xd = x[q], yd = y[q];
        x[q] = cc * xd - ss * yd;
        y[q] = ss * xd + cc * yd;
    }
}

template <typename T>
__device__ __forceinline__ void rotate_lds_col(T* vx, T* vy, int n, int gl, int G, double c, double s) {
    const T cc = (T)c, ss = (T)s;
    for (int r = gl; r < n; r += G) {
        const T xd = vx[r], yd = vy[r];
        vx[r] = cc * xd - ss * yd;
        vy[r] = ss * xd + cc * yd;
    }
}

// Pair with both columns in LDS (rows gl + G q); na, nb are their tracked
// squared norms (LDS, updated by lane 0 of the group).  Returns 1 if rotated.
template <typename T, int R, int G>
__device__ __forceinline__ int gpair_lds(T* __restrict__ x, T* __restrict__ y, double* na, double* nb,
                                         T* __restrict__ vx, T* __restrict__ vy, int vrows, int gl, double tol,
                                         bool f64, double th2, int& big) {
    T xr[R], yr[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        xr[q] = x[gl + G * q];
        yr[q] = y[gl + G * q];
    }
    const double a = *na, b = *nb;
    const double g = group_sum<G>(partial_dot<T, R>(xr, yr, f64));
    big += !(g * g <= th2 * (a * b));  // a NaN counts as large: never converged
    double c, s, t;
    if (!rotation(a, b, g, tol, c, s, t)) return 0;
    rotate_regs<T, R>(xr, yr, c, s);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        x[gl + G * q] = xr[q];
        y[gl + G * q] = yr[q];
    }
    if (vrows) rotate_lds_col<T>(vx, vy, vrows, gl, G, c, s);
    if (gl == 0) {
        *na = a - t * g;
        *nb = b + t * g;
    }
    return 1;
}


// Team-kernel columns carry RT values per lane: the first R are the rows of A
// (row gl + G q), the others (RT > R when V is accumulated) the rows of V
// (row gl + G (q - R)).  Inner products and norms use the A rows; rotations
// act on the whole column, so V follows every rotation of A.
//
// Kept-column mode (keep2 >= 0): a pair whose two squared norms are both
// <= keep2 (a "rest" pair) is skipped before any load or product.  ev counts
// the pairs evaluated, prog those with cosine > 1e-2 (the mode's measure of
// progress).
template <typename T, int R, int RT, int G>
__device__ __forceinline__ int tpair_lds(T* __restrict__ x, T* __restrict__ y, double* na, double* nb, int gl,
                                         double tol, bool f64, double th2, double keep2, int& big, int& ev,
                                         int& prog) {
    const double a = *na, b = *nb;
    if (a <= keep2 && b <= keep2) return 0;  // (a NaN norm makes a kept pair)
    ++ev;
    T xr[RT], yr[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        xr[q] = x[gl + G * q];
        yr[q] = y[gl + G * q];
    }
    const double g = group_dot<T, R, G>(xr, yr, f64);
    big += !(g * g <= th2 * (a * b));  // a NaN counts as large: never converged
    prog += !(g * g <= 1e-4 * (a * b));
    double c, s, t;
    if (!rotation(a, b, g, tol, c, s, t)) return 0;
    rotate_regs<T, RT>(xr, yr, c, s);
#pragma unroll
    for (int q = 0; q < RT; ++q) {
        x[gl + G * q] = xr[q];
        y[gl + G * q] = yr[q];
    }
    if (gl == 0) {
        *na = a - t * g;
        *nb = b + t * g;
    }
    return 1;
}

// Pair with x in registers (squared norm na, uniform in the group) and y in LDS.
// keep2, ev and prog as for tpair_lds.
template <typename T, int R, int RT, int G>
__device__ __forceinline__ int tpair_reg(T (&xr)[RT], double& na, T* __restrict__ y, double* nb, int gl,
                                         double tol, bool f64, double th2, double keep2, int& big, int& ev,
                                         int& prog) {
    const double b = *nb;
    const double a = na;
    if (a <= keep2 && b <= keep2) return 0;
    ++ev;
    T yr[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) yr[q] = y[gl + G * q];
    const double g = group_dot<T, R, G>(xr, yr, f64);
    big += !(g * g <= th2 * (a * b));  // a NaN counts as large: never converged
    prog += !(g * g <= 1e-4 * (a * b));
    double c, s, t;
    if (!rotation(a, b, g, tol, c, s, t)) return 0;
    rotate_regs<T, RT>(xr, yr, c, s);
#pragma unroll
    for (int q = 0; q < RT; ++q) y[gl + G * q] = yr[q];
    na = a - t * g;
    if (gl == 0) *nb = b + t * g;
    return 1;
}

// Two independent pairs (x1, y1) and (x2, y2), all in registers, with squared
// norms n1, m1, n2, m2 (uniform in the group); v1, v2 say whether each pair is
// real (padding columns are skipped).  The two dot products, reductions and
// angles are independent chains, which the wavefront interleaves.  A pair
// that needs no rotation gets c = 1, s = 0 (exact identity).
template <typename T, int R, int G>
__device__ __forceinline__ int gpair2(T (&x1)[R], double& n1, T (&y1)[R], double& m1, T (&x2)[R], double& n2,
                                      T (&y2)[R], double& m2, bool v1, bool v2, double tol, bool f64, double th2,
                                      int& big) {
    const double g1 = group_sum<G>(partial_dot<T, R>(x1, y1, f64));
    const double g2 = group_sum<G>(partial_dot<T, R>(x2, y2, f64));
    big += (v1 && !(g1 * g1 <= th2 * (n1 * m1))) + (v2 && !(g2 * g2 <= th2 * (n2 * m2)));
    const bool r1 = v1 && needs_rotation(n1, m1, g1, tol);
    const bool r2 = v2 && needs_rotation(n2, m2, g2, tol);
    if (r1 || r2) {
        double c1, s1, t1, c2, s2, t2;
        // benign arguments for a pair that does not rotate; its results are replaced below
        rotation_angle(r1 ? n1 : 1.0, r1 ? m1 : 2.0, r1 ? g1 : 1.0, c1, s1, t1);
        rotation_angle(r2 ? n2 : 1.0, r2 ? m2 : 2.0, r2 ? g2 : 1.0, c2, s2, t2);
        c1 = r1 ? c1 : 1.0; s1 = r1 ? s1 : 0.0; t1 = r1 ? t1 : 0.0;
        c2 = r2 ? c2 : 1.0; s2 = r2 ? s2 : 0.0; t2 = r2 ? t2 : 0.0;
        rotate_regs<T, R>(x1, y1, c1, s1);
        rotate_regs<T, R>(x2, y2, c2, s2);
        n1 -= t1 * g1; m1 += t1 * g1;
        n2 -= t2 * g2; m2 += t2 * g2;
    }
    return (int)r1 + (int)r2;
}

// Squared norm of an LDS column (rows gl + G q), reduced over the group.
template <typename T, int R, int G>
__device__ __forceinline__ double lds_col_norm(const T* __restrict__ x, int gl) {
    T xr[R];
#pragma unroll
    for (int q = 0; q < R; ++q) xr[q] = x[gl + G * q];
    return group_sum<G>(partial_norm<T, R>(xr));
}

// Element (r, c) of slice k's tall matrix in the source tensor.
template <typename T>
__device__ __forceinline__ T src_at(const JacobiJob& J, int k, int r, int c) {
    return ((const T*)J.src)[(int64_t)k * J.src_ss + (int64_t)r * J.src_rs + (int64_t)c * J.src_cs];
}

// Sum of one value per lane group (uniform within the group) over the block.
__device__ __forceinline__ int block_sum_groups(int v, int gl, int* s_scratch) {
    if (threadIdx.x == 0) *s_scratch = 0;
    __syncthreads();
    if (gl == 0 && v) atomicAdd(s_scratch, v);
    __syncthreads();
    const int tot = *s_scratch;
    __syncthreads();
    return tot;
}

__device__ __forceinline__ void record_slice(const JacobiJob& J, int k, int sweeps, int executed, Ctrl* ctrl) {
    J.sweeps[k] = sweeps;
    if (sweeps < 0) {
        if (!J.keep) atomicOr(&ctrl->status, kStNoConv);  // kept-column mode: the certificate decides
    } else {
        atomicMax(&ctrl->max_sweeps, sweeps);
    }
    atomicAdd(&ctrl->slice_sweeps, (unsigned long long)executed);
}

// ---------------------------------------------------------------------------
// Resident kernel.  LDS: pp columns of ldl = R*G rows of A, then (with V) pp
// columns of ldv rows (ldv >= p).
// ---------------------------------------------------------------------------
template <typename T, int R, int G, bool WV>
__device__ void resident_task(const JacobiJob& J, int k, int max_sweeps, Ctrl* ctrl, T* lds, int* s_scratch,
                              double* s_nrm) {
    constexpr int ldl = R * G + kLdsPad;
    const int m = J.m, p = J.p, ldv = J.ldv;
    const int pp = p + (p & 1);
    T* As = lds;
    T* Vs = lds + (int64_t)pp * ldl;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int grp = tid / G, gl = tid % G, ngrp = nth / G;

    if (J.src_rs == 1) {
        for (int e = tid; e < pp * ldl; e += nth) {
            const int c = e / ldl, r = e - c * ldl;
            As[e] = (c < p && r < m) ? src_at<T>(J, k, r, c) : (T)0;
        }
    } else {  // transposed source: walk columns fastest for contiguous reads
        for (int e = tid; e < pp * ldl; e += nth) {
            const int r = e / pp, c = e - r * pp;
            As[c * ldl + r] = (c < p && r < m) ? src_at<T>(J, k, r, c) : (T)0;
        }
    }
    if (WV) {
        const T* Vg0 = (const T*)J.V + (int64_t)k * p * p;
        for (int e = tid; e < pp * ldv; e += nth) {
            const int c = e / ldv, r = e - c * ldv;
            T v = (r == c) ? (T)1 : (T)0;
            if (J.vinit) v = (c < p && r < p) ? Vg0[(int64_t)c * p + r] : (T)0;  // warm start
            Vs[e] = v;
        }
    }
    __syncthreads();

    const double tol = J.tol;
    int sweeps = -1, executed = 0;
    const bool refine = J.refine64 != 0;
    for (int sw = 0; sw < max_sweeps + (refine ? 1 : 0); ++sw) {
        const bool f64 = refine && sw == max_sweeps;  // reached only through the refinement path
        const double tl = f64 ? (double)m * Unit<double>::v : tol;
        int rot = 0, big = 0;
        ++executed;
        // exact squared column norms at the start of each sweep, tracked after
        for (int c = grp; c < p; c += ngrp) {
            const double nn = lds_col_norm<T, R, G>(As + c * ldl, gl);
            if (gl == 0) s_nrm[c] = nn;
        }
        __syncthreads();
        for (int s = 0; s < pp - 1; ++s) {
            for (int q = grp; q < pp / 2; q += ngrp) {
                int i, j;
                rr_pair(s, q, pp, i, j);
                if (j < p)
                    rot += gpair_lds<T, R, G>(As + i * ldl, As + j * ldl, s_nrm + i, s_nrm + j,
                                              WV ? Vs + i * ldv : nullptr, WV ? Vs + j * ldv : nullptr, WV ? p : 0,
                                              gl, tl, f64, J.skip2, big);
            }
            __syncthreads();
        }
        const int tot = block_sum_groups(rot, gl, s_scratch);
        const int btot = block_sum_groups(big, gl, s_scratch);
        if (f64) break;
        if (tot == 0 || btot == 0) {
            sweeps = sw + 1;
            if (!refine) break;
            sw = max_sweeps - 1;  // one more sweep, with FP64 inner products and angles
        }
    }
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    for (int e = tid; e < p * m; e += nth) {
        const int c = e / m, r = e - c * m;
        Ag[e] = As[c * ldl + r];
    }
    if (WV) {
        T* Vg = (T*)J.V + (int64_t)k * p * p;
        for (int e = tid; e < p * p; e += nth) {
            const int c = e / p, r = e - c * p;
            Vg[e] = Vs[c * ldv + r];
        }
    }
    if (tid == 0) record_slice(J, k, sweeps, executed, ctrl);
}

#define TSVD_DISPATCH_RG(J, CALL)                          \
    do {                                                   \
        if ((J).G == 16) {                                 \
            switch ((J).R) {                               \
                case 4: CALL(4, 16); break;                \
                case 8: CALL(8, 16); break;                \
                case 12: CALL(12, 16); break;              \
                default: CALL(16, 16); break;              \
            }                                              \
        } else {                                           \
            switch ((J).R) {                               \
                case 4: CALL(4, 32); break;                \
                case 8: CALL(8, 32); break;                \
                case 12: CALL(12, 32); break;              \
                default: CALL(16, 32); break;              \
            }                                              \
        }                                                  \
    } while (0)

template <typename T, bool WV>
__global__ __launch_bounds__(1024) void k_jacobi_resident(JacobiJob job1, const JacobiJob* __restrict__ jobs,
                                                          const int* __restrict__ task_job,
                                                          const int* __restrict__ task_slice, int ntasks,
                                                          int max_sweeps, Ctrl* ctrl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_scratch;
    __shared__ double s_nrm[kMaxRows];
    T* lds = (T*)smem_raw;
    for (int t = blockIdx.x; t < ntasks; t += gridDim.x) {
        // one tensor: the job travels by value and task t is slice t
        const JacobiJob J = jobs ? jobs[task_job[t]] : job1;
        const int k = jobs ? task_slice[t] : t;
        Ctrl* jc = J.ctrl ? J.ctrl : ctrl;
#define TSVD_RES_CALL(RR, GG) resident_task<T, RR, GG, WV>(J, k, max_sweeps, jc, lds, &s_scratch, s_nrm)
        TSVD_DISPATCH_RG(J, TSVD_RES_CALL);
#undef TSVD_RES_CALL
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Team kernel.
// ---------------------------------------------------------------------------
struct TeamState {
    int* bar;       // this team's W barrier flags (one per workgroup)
    int passed;     // barriers passed so far by this workgroup
    int W;
    int spin_limit;
    Ctrl* ctrl;
    int rank;       // this workgroup's flag
    int* blk;       // this team's block flags (nb): the step at which each block was last released
    int steps;      // block-pair steps finished so far by this workgroup
};

// XCD (accelerator complex die) of the executing workgroup: hardware register
// XCC_ID, read with s_getreg_b32 (id 20, bits [3:0]).
__device__ __forceinline__ int xcc_id() { return __builtin_amdgcn_s_getreg((15 << 11) | 20) & 0xF; }

// Team barrier.  Each wavefront first waits for its own global stores to be
// acknowledged by the L2 (vmcnt(0)); then thread 0 writes the number of
// barriers this workgroup has passed to its own flag with an ordinary store
// (through to the L2), and lanes 0..W-1 of wavefront 0 poll the W flags of the
// team together, with a bounded spin, until every one has reached that count.
// All workgroups of a team run on one XCD and so share one L2: the flags and
// the exchanged blocks are there as soon as the stores are acknowledged, and
// the polls and block loads bypass the L1 (ld_team), so neither a release
// write-back of the L2 nor an acquire invalidation is needed, and no
// device-scope atomic either.  Returns false when the wait gave up.
__device__ bool team_barrier(TeamState& ts, int* s_flag) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's stores are complete
    __syncthreads();
    ts.passed += 1;
    if (threadIdx.x < kWave) {
        if (threadIdx.x == 0) *s_flag = 0;
        if (ts.W > 1) {
            if (threadIdx.x == 0) {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __hip_atomic_store(ts.bar + ts.rank, ts.passed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            const int lane = threadIdx.x;
            int it = 0;
            for (;;) {
                const int f = lane < ts.W ? ld_team(ts.bar + lane) : ts.passed;
                if (__all(f >= ts.passed)) break;
                if (++it > ts.spin_limit) {
                    if (lane == 0) {
                        atomicOr(&ts.ctrl->status, kStTimeout);
                        *s_flag = 1;
                    }
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
    }
    __syncthreads();
    // s_flag is next written by thread 0 after the workgroup barrier that opens the
    // next team barrier, so every thread has read it by then
    return *s_flag == 0;
}

// Point-to-point hand-over of blocks between the steps of a sweep.  A block
// goes from the workgroup that held it in one step to the one that holds it
// in the next, so a workgroup waits only for the two previous holders of its
// blocks instead of the whole team.  Release: every wavefront's stores are
// acknowledged by the L2 (vmcnt(0)), then thread 0 writes the step number to
// both block flags with ordinary stores.  Wait: lanes 0 and 1 of wavefront 0
// poll the two flags (L1-bypassing loads, bounded spin).  The last step of a
// sweep still ends at the full team barrier, which also publishes the
// rotation counts that decide convergence.
__device__ void team_release_blocks(TeamState& ts, int BI, int BJ, int step) {
    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): this wavefront's stores are complete
    __syncthreads();
    if (ts.W > 1 && threadIdx.x == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __hip_atomic_store(ts.blk + BI, step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        __hip_atomic_store(ts.blk + BJ, step, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    }
}

__device__ bool team_wait_blocks(TeamState& ts, int BI, int BJ, int step, int* s_flag) {
    if (ts.W == 1) return true;  // this workgroup stored them itself (release waited for the stores)
    if (threadIdx.x < kWave) {
        const int lane = threadIdx.x;
        if (lane == 0) *s_flag = 0;
        int it = 0;
        for (;;) {
            const int f = lane == 0 ? ld_team(ts.blk + BI) : lane == 1 ? ld_team(ts.blk + BJ) : step;
            if (__all(f >= step)) break;
            if (++it > ts.spin_limit) {
                if (lane == 0) {
                    atomicOr(&ts.ctrl->status, kStTimeout);
                    *s_flag = 1;
                }
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    return *s_flag == 0;
}

// Load b columns of block `blk` into LDS (ld ldl); from the source tensor on
// the first step of the first sweep, else from A.  Zero padding beyond m / p.
// Column squared norms go to nrm[] (LDS), except from a transposed source,
// whose loads do not follow the lane groups (the caller takes those from LDS).
template <typename T, int R, int G, bool WV>
__device__ __forceinline__ void team_load_block(const JacobiJob& J, int k, int blk, bool first, T* As,
                                                double* nrm) {
    constexpr int RT = WV ? 2 * R : R;
    constexpr int ldl = RT * G + kLdsPad;
    const int m = J.m, p = J.p, b = J.b;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int grp = tid / G, gl = tid % G, c = blk * b + grp;
    const T* Ag = (const T*)J.A + (int64_t)k * m * p;
    if (first && J.src_rs != 1) {
        // transposed source: consecutive lanes take consecutive columns (contiguous in memory)
        for (int e = tid; e < b * (R * G); e += nth) {
            const int r = e / b, cl = e - r * b, cc = blk * b + cl;
            As[cl * ldl + r] = (cc < p && r < m) ? src_at<T>(J, k, r, cc) : (T)0;
        }
    } else {
        // group g (G lanes) takes column g of the block, rows gl + G q: R loads in flight per lane
        T v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = gl + G * q;
            v[q] = (T)0;
            if (c < p && r < m) v[q] = first ? src_at<T>(J, k, r, c) : ld_team(Ag + (int64_t)c * m + r);
        }
#pragma unroll
        for (int q = 0; q < R; ++q) As[grp * ldl + gl + G * q] = v[q];
        // the column's squared norm from the loaded values (same order as lds_col_norm)
        const double nn = group_sum<G>(partial_norm<T, R>(v));
        if (gl == 0) nrm[grp] = nn;
    }
    if (WV) {
        // V rows below the A rows: the identity, the caller's V (warm start) or the work array
        const T* Vg = (const T*)J.V + (int64_t)k * p * p;
        T v[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = gl + G * q;
            v[q] = (T)0;
            if (c < p && r < p) {
                if (!first) v[q] = ld_team(Vg + (int64_t)c * p + r);
                else v[q] = J.vinit ? Vg[(int64_t)c * p + r] : (T)(r == c ? 1 : 0);
            }
        }
#pragma unroll
        for (int q = 0; q < R; ++q) As[grp * ldl + gl + G * (R + q)] = v[q];
    }
}

// Write a block back to the work arrays (group g stores column g).
template <typename T, int R, int G, bool WV>
__device__ __forceinline__ void team_store_block(const JacobiJob& J, int k, int blk, const T* As) {
    constexpr int RT = WV ? 2 * R : R;
    constexpr int ldl = RT * G + kLdsPad;
    const int m = J.m, p = J.p, b = J.b;
    const int grp = threadIdx.x / G, gl = threadIdx.x % G, c = blk * b + grp;
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    T v[RT];
#pragma unroll
    for (int q = 0; q < RT; ++q) v[q] = As[grp * ldl + gl + G * q];
    if (c < p) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = gl + G * q;
            if (r < m) Ag[(int64_t)c * m + r] = v[q];
        }
        if (WV) {
            T* Vg = (T*)J.V + (int64_t)k * p * p;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int r = gl + G * q;
                if (r < p) Vg[(int64_t)c * p + r] = v[R + q];
            }
        }
    }
}

// Load a block of B = 2 ng columns into LDS: group g takes columns 2g, 2g + 1.
template <typename T, int R, int G>
__device__ __forceinline__ void team_load_block2(const JacobiJob& J, int k, int blk, bool first, T* As) {
    constexpr int ldl = R * G + kLdsPad;
    const int m = J.m, p = J.p, B = J.b;
    const int tid = threadIdx.x, nth = blockDim.x;
    const T* Ag = (const T*)J.A + (int64_t)k * m * p;
    if (first && J.src_rs != 1) {
        // transposed source: consecutive lanes take consecutive columns (contiguous in memory)
        for (int e = tid; e < B * ldl; e += nth) {
            const int r = e / B, cl = e - r * B, c = blk * B + cl;
            As[cl * ldl + r] = (c < p && r < m) ? src_at<T>(J, k, r, c) : (T)0;
        }
        return;
    }
    const int grp = tid / G, gl = tid % G, ca = blk * B + 2 * grp, cb = ca + 1;
    T va[R], vb[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = gl + G * q;
        va[q] = (T)0;
        vb[q] = (T)0;
        if (r < m) {
            if (ca < p) va[q] = first ? src_at<T>(J, k, r, ca) : ld_team(Ag + (int64_t)ca * m + r);
            if (cb < p) vb[q] = first ? src_at<T>(J, k, r, cb) : ld_team(Ag + (int64_t)cb * m + r);
        }
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        As[(2 * grp) * ldl + gl + G * q] = va[q];
        As[(2 * grp + 1) * ldl + gl + G * q] = vb[q];
    }
}

// Store a block of B = 2 ng columns: group g writes columns 2g, 2g + 1.
template <typename T, int R, int G>
__device__ __forceinline__ void team_store_block2(const JacobiJob& J, int k, int blk, const T* As) {
    constexpr int ldl = R * G + kLdsPad;
    const int m = J.m, p = J.p, B = J.b;
    const int grp = threadIdx.x / G, gl = threadIdx.x % G, ca = blk * B + 2 * grp, cb = ca + 1;
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    T va[R], vb[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        va[q] = As[(2 * grp) * ldl + gl + G * q];
        vb[q] = As[(2 * grp + 1) * ldl + gl + G * q];
    }
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int r = gl + G * q;
        if (r < m) {
            if (ca < p) Ag[(int64_t)ca * m + r] = va[q];
            if (cb < p) Ag[(int64_t)cb * m + r] = vb[q];
        }
    }
}

// Write a block back to the work array (group g stores column g).
template <typename T, int R, int G, bool WV>
__device__ __forceinline__ void team_store_block(const JacobiJob& J, int k, int blk, const T* As, const T* Vs) {
    constexpr int ldl = R * G + kLdsPad;
    const int m = J.m, p = J.p, b = J.b, ldv = J.ldv;
    const int tid = threadIdx.x, nth = blockDim.x;
    const int grp = tid / G, gl = tid % G, c = blk * b + grp;
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    T v[R];
#pragma unroll
    for (int q = 0; q < R; ++q) v[q] = As[grp * ldl + gl + G * q];
    if (c < p) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = gl + G * q;
            if (r < m) Ag[(int64_t)c * m + r] = v[q];
        }
    }
    if (WV) {
        T* Vg = (T*)J.V + (int64_t)k * p * p;
        for (int e = tid; e < b * p; e += nth) {
            const int cl = e / p, r = e - cl * p, cc = blk * b + cl;
            if (cc < p) Vg[(int64_t)cc * p + r] = Vs[cl * ldv + r];
        }
    }
}

// One slice by one team.  Returns false if a barrier timed out.
template <typename T, int R, int G, bool WV>
__device__ bool team_task(const JacobiJob& J, int k, int rank, TeamState& ts, int max_sweeps, T* lds,
                          int* s_scratch, int* s_flag, double* nI, double* nJ) {
    constexpr int RT = WV ? 2 * R : R;     // A rows, then V rows, per lane
    constexpr int ldl = RT * G + kLdsPad;
    const int m = J.m, p = J.p, b = J.b, nb = J.nb;
    const int tid = threadIdx.x, grp = tid / G, gl = tid % G;  // one lane group per I column (b groups)
    T* Is = lds;                           // b columns x ldl (first step of a sweep)
    T* Js = lds + (int64_t)b * ldl;        // b columns x ldl
    const double tol = J.tol;
    const bool refine = J.refine64 != 0;
    int sweeps = -1, executed = 0;
    int* rot_g = J.rot + (int64_t)k * kRotStride;
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    T* Vg = WV ? (T*)J.V + (int64_t)k * p * p : nullptr;
    // a slice already done (uniform over the team: every member reads the same flag)
    if (J.skip && J.skip[k]) return true;
    // kept-column mode, until the slice turns into the full iteration (uniform
    // over the team: decided from the slice's counters after a team barrier)
    int keep = J.keep;
    double kt2 = J.keep2;
    if (keep && J.keep_sched) {
        const double t = J.keep_sched[ts.ctrl->iter];
        kt2 = t * t;
    }
    int slow = 0;  // consecutive kept-column sweeps of slow progress
    const bool final_sweep = refine || keep;
    for (int sw = 0; sw < max_sweeps + (final_sweep ? 1 : 0); ++sw) {
        const bool fin = final_sweep && sw == max_sweeps;
        const bool f64 = refine && fin;
        const double keep2 = keep ? kt2 : -1.0;
        const double tl = f64 ? (double)m * Unit<double>::v : tol;
        int rot = 0, big = 0, ev = 0, prog = 0;
        ++executed;
        for (int s = 0; s < nb - 1; ++s) {
            const bool last = (s == nb - 2);
            for (int q = rank; q < nb / 2; q += ts.W) {
                int BI, BJ;
                rr_pair(s, q, nb, BI, BJ);
                // the first step of a sweep follows a full team barrier (or reads the source)
                if (s > 0 && !team_wait_blocks(ts, BI, BJ, ts.steps, s_flag)) return false;
                const bool first = (sw == 0 && s == 0);
                const int ci = BI * b + grp;  // this group's I column
                const int cs = ci < p ? ci : 0;
                T xr[RT];
                double na = 0.0;
                if (s != 0) {
                    // this group's I column comes from the work arrays; its loads are issued
                    // first so that they overlap with the J block's (the clamped column keeps
                    // every load in bounds; rows beyond m, or p for V, read as zero)
#pragma unroll
                    for (int q2 = 0; q2 < R; ++q2) {
                        const int r = gl + G * q2;
                        xr[q2] = (T)0;
                        if (r < m) xr[q2] = ld_team(Ag + (int64_t)cs * m + r);
                        if (WV) {
                            xr[R + q2] = (T)0;
                            if (r < p) xr[R + q2] = ld_team(Vg + (int64_t)cs * p + r);
                        }
                    }
                }
                team_load_block<T, R, G, WV>(J, k, BJ, first, Js, nJ);
                if (s == 0) team_load_block<T, R, G, WV>(J, k, BI, first, Is, nI);
                __syncthreads();
                if (first && J.src_rs != 1) {
                    const double nn = lds_col_norm<T, R, G>(Js + grp * ldl, gl);
                    const double ni = lds_col_norm<T, R, G>(Is + grp * ldl, gl);
                    if (gl == 0) {
                        nJ[grp] = nn;
                        nI[grp] = ni;
                    }
                    __syncthreads();
                }
                if (s == 0) {
                    // pairs inside each block: b-1 rounds, b/2 pairs per block per round
                    for (int r = 0; r < b - 1; ++r) {
                        const int half = grp < b / 2 ? 0 : 1;
                        int i, j;
                        rr_pair(r, grp - half * (b / 2), b, i, j);
                        const int blk = half ? BJ : BI;
                        T* base = half ? Js : Is;
                        double* nb_ = half ? nJ : nI;
                        if (blk * b + j < p)
                            rot += tpair_lds<T, R, RT, G>(base + i * ldl, base + j * ldl, nb_ + i, nb_ + j, gl, tl,
                                                          f64, J.skip2, keep2, big, ev, prog);
                        __syncthreads();
                    }
#pragma unroll
                    for (int q2 = 0; q2 < RT; ++q2) xr[q2] = Is[grp * ldl + gl + G * q2];
                    na = nI[grp];
                } else {
                    na = group_sum<G>(partial_norm<T, R>(xr));
                }
                // cross pairs.  The J block is cut into sub-blocks of gw = 64 / G columns, one
                // per wavefront of gw lane groups.  In super-round r wavefront w owns sub-block
                // (w + r) mod nw, and its group u pairs with column (u + v) mod gw of it in
                // sub-round v.  Between sub-rounds a J column passes between groups of one
                // wavefront, whose LDS accesses complete in program order, so only the
                // super-rounds end at a workgroup barrier.
                {
                    constexpr int gw = kWave / G;
                    const int nw = b / gw, w = grp / gw, u = grp - w * gw;
                    int sb = w;
                    for (int r = 0; r < nw; ++r, sb = (sb + 1 == nw) ? 0 : sb + 1) {
#pragma unroll
                        for (int v = 0; v < gw; ++v) {
                            const int j = sb * gw + ((u + v) & (gw - 1));
                            if (ci < p && BJ * b + j < p)
                                rot += tpair_reg<T, R, RT, G>(xr, na, Js + j * ldl, nJ + j, gl, tl, f64, J.skip2,
                                                              keep2, big, ev, prog);
                            // keeps the compiler from moving the next sub-round's LDS reads
                            // above this one's writes (no instruction is emitted)
                            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        }
                        __syncthreads();
                    }
                }
                if (ci < p) {
#pragma unroll
                    for (int q2 = 0; q2 < R; ++q2) {
                        const int r = gl + G * q2;
                        if (r < m) Ag[(int64_t)ci * m + r] = xr[q2];
                        if (WV && r < p) Vg[(int64_t)ci * p + r] = xr[R + q2];
                    }
                }
                team_store_block<T, R, G, WV>(J, k, BJ, Js);
                // the LDS blocks are reloaded next by this loop or after the team barrier,
                // and both the release and the team barrier begin with a workgroup barrier
                if (!last) team_release_blocks(ts, BI, BJ, ts.steps + 1);
                else if (q + ts.W < nb / 2) __syncthreads();
            }
            ts.steps += 1;
            if (last) {
                const int tot = block_sum_groups(rot, gl, s_scratch);
                const int btot = block_sum_groups(big, gl, s_scratch);
                if (tid == 0 && tot) atomicAdd(rot_g + sw, tot);
                if (tid == 0 && btot) atomicAdd(rot_g + kMaxSweeps + sw, btot);
                if (keep) {
                    const int etot = block_sum_groups(ev, gl, s_scratch);
                    const int ptot = block_sum_groups(prog, gl, s_scratch);
                    if (tid == 0 && etot) {
                        atomicAdd(&ts.ctrl->pairs, (unsigned long long)etot);
                        atomicAdd(rot_g + 2 * kMaxSweeps + sw, etot);
                    }
                    if (tid == 0 && ptot) atomicAdd(rot_g + 3 * kMaxSweeps + sw, ptot);
                }
                if (!team_barrier(ts, s_flag)) return false;
            }
        }
        if (fin) break;
        const int total = __hip_atomic_load(rot_g + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int large = __hip_atomic_load(rot_g + kMaxSweeps + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (keep && sw >= 1 && !(total == 0 || large == 0)) {
            // Signs that the kept columns will not settle soon, or that the columns
            // left below tau sit near it, beyond what the certificate can clear
            // (past the first sweep, which starts from the input's columns): a
            // sweep that still evaluated over 40% of all pairs (a large kept set);
            // a sweep with an unchanged kept set (the same number of pairs
            // evaluated as the one before) whose pairs with cosine > 1e-2 fell by
            // less than a factor 0.5, or two in a row by less than 0.35 (a
            // continuous spectrum through tau); the sweep limit of the mode.  The
            // slice then continues as the full iteration (this sweep's counts
            // covered the kept pairs only, so they decide nothing).
            auto ld = [&](int seg, int w) {
                return __hip_atomic_load(rot_g + seg * kMaxSweeps + w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            };
            const int evs = ld(2, sw), evp = ld(2, sw - 1), pg = ld(3, sw), pgp = ld(3, sw - 1);
            const bool stable = evs == evp && pg > 0;
            slow = (stable && pg > 0.35 * pgp) ? slow + 1 : 0;
            if (2.0 * evs > 0.4 * (double)p * (p - 1) || (stable && pg > 0.5 * pgp) || slow >= 2 ||
                sw + 1 >= kKeepMaxSweeps) {
                keep = 0;
                continue;
            }
        }
        if (total == 0 || large == 0) {
            sweeps = sw + 1;
            if (!final_sweep || (!keep && !refine)) break;
            sw = max_sweeps - 1;
        }
    }
    if (tid == 0 && rank == 0) {
        if (J.keep && !keep && sweeps >= 0) J.full[k] = 1;
        record_slice(J, k, sweeps, executed, ts.ctrl);
    }
    return true;
}

// Team task with two columns per lane group (no V).  Blocks are B = J.b
// columns wide and a workgroup has ng = B / 2 groups.  The I block lives in
// registers, columns 2g and 2g + 1 in group g; the J block in LDS.  A cross
// round gives group g the J columns 2j, 2j + 1 (j = (g + r) mod ng) and does
// the pairs (x1, y1), (x2, y2) together, then (x1, y2), (x2, y1): two
// independent rotations at a time, and each J column read from LDS serves two
// pairs (half the LDS traffic of one column per group).  The first step of a
// sweep also pairs the columns inside each block: B - 1 rounds, group g takes
// pair g of the I block and pair g of the J block.
template <typename T, int R, int G>
__device__ bool team_task_k2(const JacobiJob& J, int k, int rank, TeamState& ts, int max_sweeps, T* lds,
                             int* s_scratch, int* s_flag, double* nI, double* nJ) {
    constexpr int ldl = R * G + kLdsPad;
    const int m = J.m, p = J.p, B = J.b, nb = J.nb, ng = J.b / 2;
    const int tid = threadIdx.x, grp = tid / G, gl = tid % G;
    T* Is = lds;                        // B columns x ldl (first step of a sweep)
    T* Js = lds + (int64_t)B * ldl;     // B columns x ldl
    const double tol = J.tol;
    const bool refine = J.refine64 != 0;
    int sweeps = -1, executed = 0;
    int* rot_g = J.rot + (int64_t)k * kRotStride;
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    for (int sw = 0; sw < max_sweeps + (refine ? 1 : 0); ++sw) {
        const bool f64 = refine && sw == max_sweeps;
        const double tl = f64 ? (double)m * Unit<double>::v : tol;
        int rot = 0, big = 0;
        ++executed;
        for (int s = 0; s < nb - 1; ++s) {
            for (int q = rank; q < nb / 2; q += ts.W) {
                int BI, BJ;
                rr_pair(s, q, nb, BI, BJ);
                const bool first = (sw == 0 && s == 0);
                const int c1 = BI * B + 2 * grp, c2 = c1 + 1;  // this group's I columns
                T x1[R], x2[R];
                double n1 = 0.0, n2 = 0.0;
                if (s != 0) {
                    // the I columns come from the work array; their loads are issued first
                    const T* xs1 = Ag + (int64_t)(c1 < p ? c1 : 0) * m;
                    const T* xs2 = Ag + (int64_t)(c2 < p ? c2 : 0) * m;
#pragma unroll
                    for (int q2 = 0; q2 < R; ++q2) {
                        const int r = gl + G * q2;
                        x1[q2] = (T)0;
                        x2[q2] = (T)0;
                        if (r < m) {
                            x1[q2] = ld_team(xs1 + r);
                            x2[q2] = ld_team(xs2 + r);
                        }
                    }
                }
                team_load_block2<T, R, G>(J, k, BJ, first, Js);
                if (s == 0) team_load_block2<T, R, G>(J, k, BI, first, Is);
                __syncthreads();
                {
                    const double a0 = lds_col_norm<T, R, G>(Js + (2 * grp) * ldl, gl);
                    const double a1 = lds_col_norm<T, R, G>(Js + (2 * grp + 1) * ldl, gl);
                    if (gl == 0) { nJ[2 * grp] = a0; nJ[2 * grp + 1] = a1; }
                    if (s == 0) {
                        const double b0 = lds_col_norm<T, R, G>(Is + (2 * grp) * ldl, gl);
                        const double b1 = lds_col_norm<T, R, G>(Is + (2 * grp + 1) * ldl, gl);
                        if (gl == 0) { nI[2 * grp] = b0; nI[2 * grp + 1] = b1; }
                    }
                }
                __syncthreads();
                if (s == 0) {
                    // pairs inside each block: B - 1 rounds of ng pairs per block
                    for (int r = 0; r < B - 1; ++r) {
                        int i1, j1;
                        rr_pair(r, grp, B, i1, j1);  // pair grp of this round, in both blocks
                        const bool vI = BI * B + j1 < p, vJ = BJ * B + j1 < p;
                        T a[R], b[R], c[R], d[R];
#pragma unroll
                        for (int q2 = 0; q2 < R; ++q2) {
                            const int rr = gl + G * q2;
                            a[q2] = Is[i1 * ldl + rr];
                            b[q2] = Is[j1 * ldl + rr];
                            c[q2] = Js[i1 * ldl + rr];
                            d[q2] = Js[j1 * ldl + rr];
                        }
                        double na = nI[i1], nbb = nI[j1], nc = nJ[i1], nd = nJ[j1];
                        rot += gpair2<T, R, G>(a, na, b, nbb, c, nc, d, nd, vI, vJ, tl, f64, J.skip2, big);
#pragma unroll
                        for (int q2 = 0; q2 < R; ++q2) {
                            const int rr = gl + G * q2;
                            Is[i1 * ldl + rr] = a[q2];
                            Is[j1 * ldl + rr] = b[q2];
                            Js[i1 * ldl + rr] = c[q2];
                            Js[j1 * ldl + rr] = d[q2];
                        }
                        if (gl == 0) {
                            nI[i1] = na; nI[j1] = nbb;
                            nJ[i1] = nc; nJ[j1] = nd;
                        }
                        __syncthreads();
                    }
#pragma unroll
                    for (int q2 = 0; q2 < R; ++q2) {
                        x1[q2] = Is[(2 * grp) * ldl + gl + G * q2];
                        x2[q2] = Is[(2 * grp + 1) * ldl + gl + G * q2];
                    }
                    n1 = nI[2 * grp];
                    n2 = nI[2 * grp + 1];
                } else {
                    n1 = group_sum<G>(partial_norm<T, R>(x1));
                    n2 = group_sum<G>(partial_norm<T, R>(x2));
                }
                // cross pairs: ng rounds; group g meets J columns 2j, 2j + 1, j = (g + r) mod ng
                const bool u1 = c1 < p, u2 = c2 < p;
                int j = grp;
                for (int r = 0; r < ng; ++r, j = (j + 1 == ng) ? 0 : j + 1) {
                    T y1[R], y2[R];
#pragma unroll
                    for (int q2 = 0; q2 < R; ++q2) {
                        y1[q2] = Js[(2 * j) * ldl + gl + G * q2];
                        y2[q2] = Js[(2 * j + 1) * ldl + gl + G * q2];
                    }
                    double m1 = nJ[2 * j], m2 = nJ[2 * j + 1];
                    const bool w1 = BJ * B + 2 * j < p, w2 = BJ * B + 2 * j + 1 < p;
                    rot += gpair2<T, R, G>(x1, n1, y1, m1, x2, n2, y2, m2, u1 && w1, u2 && w2, tl, f64, J.skip2, big);
                    rot += gpair2<T, R, G>(x1, n1, y2, m2, x2, n2, y1, m1, u1 && w2, u2 && w1, tl, f64, J.skip2, big);
#pragma unroll
                    for (int q2 = 0; q2 < R; ++q2) {
                        Js[(2 * j) * ldl + gl + G * q2] = y1[q2];
                        Js[(2 * j + 1) * ldl + gl + G * q2] = y2[q2];
                    }
                    if (gl == 0) {
                        nJ[2 * j] = m1;
                        nJ[2 * j + 1] = m2;
                    }
                    __syncthreads();
                }
#pragma unroll
                for (int q2 = 0; q2 < R; ++q2) {
                    const int r = gl + G * q2;
                    if (r < m) {
                        if (u1) Ag[(int64_t)c1 * m + r] = x1[q2];
                        if (u2) Ag[(int64_t)c2 * m + r] = x2[q2];
                    }
                }
                team_store_block2<T, R, G>(J, k, BJ, Js);
                __syncthreads();
            }
            if (s == nb - 2) {
                const int tot = block_sum_groups(rot, gl, s_scratch);
                const int btot = block_sum_groups(big, gl, s_scratch);
                if (tid == 0 && tot) atomicAdd(rot_g + sw, tot);
                if (tid == 0 && btot) atomicAdd(rot_g + kMaxSweeps + sw, btot);
            }
            if (!team_barrier(ts, s_flag)) return false;
        }
        if (f64) break;
        const int total = __hip_atomic_load(rot_g + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int large = __hip_atomic_load(rot_g + kMaxSweeps + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (total == 0 || large == 0) {
            sweeps = sw + 1;
            if (!refine) break;
            sw = max_sweeps - 1;
        }
    }
    if (tid == 0 && rank == 0) record_slice(J, k, sweeps, executed, ts.ctrl);
    return true;
}

// Team formation: every workgroup takes a slot on its own XCD; once all have
// arrived, slots [W t, W t + W) of an XCD form team t there, and a workgroup
// left over on an XCD without a full team exits.  Teams are numbered across
// XCDs and take slices t, t + nteams, ...  ctl layout (ints, zeroed before the
// launch): [0, 16) slot counter per XCD, [16] arrivals, [32 + W i + r] barrier
// flag of rank r in team i, [32 + nwg + nb i + x] flag of block x in team i.
template <typename T, bool WV, int R, int G, int K>
__global__ __launch_bounds__(G == 64 ? kTeamMaxThreads64 : kTeamMaxThreads) void k_jacobi_team(JacobiJob J1, int ntasks, TeamSched sched, int max_sweeps,
                                                     Ctrl* ctrl, int spin_limit) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_scratch, s_flag, s_team, s_rank, s_nteams;
    __shared__ double s_nI[kTeamMaxThreads / 8], s_nJ[kTeamMaxThreads / 8];
    T* lds = (T*)smem_raw;
    const int W = sched.W;
    int* ctl = sched.ctl;
    if (threadIdx.x == 0) {
        const int x = xcc_id();
        const int slot = __hip_atomic_fetch_add(ctl + x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(ctl + 16, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int it = 0;
        bool ok = true;
        while (__hip_atomic_load(ctl + 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (int)gridDim.x) {
            if (++it > spin_limit) {
                atomicOr(&ctrl->status, kStTimeout);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        int before = 0, total = 0;
        for (int xx = 0; xx < 16; ++xx) {
            const int full = __hip_atomic_load(ctl + xx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) / W;
            if (xx < x) before += full;
            total += full;
        }
        const int local = slot / W;
        const int full_here = __hip_atomic_load(ctl + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) / W;
        s_team = (ok && local < full_here) ? before + local : -1;
        s_rank = slot % W;
        s_nteams = total;
        if (ok && total == 0 && blockIdx.x == 0) atomicOr(&ctrl->status, kStTimeout);
    }
    __syncthreads();
    const int team = s_team, rank = s_rank, nteams = s_nteams;
    if (team < 0) return;
    TeamState ts{ctl + 32 + team * W, 0, W, spin_limit, ctrl, rank, ctl + 32 + gridDim.x + team * J1.nb, 0};
    for (int t = team; t < ntasks; t += nteams) {
        if constexpr (K == 2) {
            static_assert(!WV, "two columns per group: no V");
            if (!team_task_k2<T, R, G>(J1, t, rank, ts, max_sweeps, lds, &s_scratch, &s_flag, s_nI, s_nJ)) return;
        } else {
            if (!team_task<T, R, G, WV>(J1, t, rank, ts, max_sweeps, lds, &s_scratch, &s_flag, s_nI, s_nJ)) return;
        }
    }
}

// ---------------------------------------------------------------------------
// Batched kernel: one persistent launch for the slices of many tensors of
// different shapes.  Workgroups take (tensor, slice) tasks from a device work
// counter in the order of the task list (the host sorts it by estimated cost,
// largest first).  A slice that fits in LDS runs the resident algorithm; a
// larger one runs the block-pair algorithm with a team of one workgroup that
// streams its block pairs through the L2 (no inter-workgroup waits).  Each
// task is done by one workgroup with a fixed algorithm, so a tensor's result
// does not depend on what else is in the batch.  512 threads; a streamed task
// needs b * G == 512.
// ---------------------------------------------------------------------------
template <typename T, int R, int G, bool WV>
__global__ __launch_bounds__(512) void k_jacobi_batched(const JacobiJob* __restrict__ jobs,
                                                        const int* __restrict__ task_job,
                                                        const int* __restrict__ task_slice, int ntasks, int* queue,
                                                        int max_sweeps, Ctrl* ctrl) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_scratch, s_flag, s_task;
    __shared__ double s_nrm[kMaxRows];
    T* lds = (T*)smem_raw;
    for (;;) {
        if (threadIdx.x == 0) s_task = atomicAdd(queue, 1);
        __syncthreads();
        const int t = s_task;
        __syncthreads();
        if (t >= ntasks) break;
        const JacobiJob J = jobs[task_job[t]];
        const int k = task_slice[t];
        Ctrl* jc = J.ctrl ? J.ctrl : ctrl;  // the job's own status and counters when it has them
        if (J.nb == 0) {
            resident_task<T, R, G, WV>(J, k, max_sweeps, jc, lds, &s_scratch, s_nrm);
        } else {
            TeamState ts{nullptr, 0, 1, 0, jc, 0, nullptr, 0};
            (void)team_task<T, R, G, WV>(J, k, 0, ts, max_sweeps, lds, &s_scratch, &s_flag, s_nrm, s_nrm + 64);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Block-Gram team kernel.  The same one-sided Jacobi method and the same team
// schedule (blocks of b = 16 columns, a round-robin tournament of block pairs
// per sweep, point-to-point hand-over between steps, a team barrier per
// sweep), but a workgroup treats its block pair X = [A_I A_J] (m x 32) as one
// unit, so that the work proportional to m runs on the matrix cores:
//   1. G = X^T X (32 x 32) on the matrix cores: BF16 hi+lo products (three,
//      the lo*lo term dropped) for the FP32 sweeps of the mixed path, FP32
//      products for the FP32 path, FP64 for FP64 data and for the mixed
//      path's final sweep (FP32 values are exact in FP64);
//   2. the step's rotations, the same pairs in the same round order as the
//      one-sided method on X, computed from G alone: with Q the product of
//      the rotations so far and K = G Q, the inner product of columns i and j
//      of X Q is q_i . k_j and the rotation of a pair acts on the columns of
//      Q and K (vectors of 32, in FP64, tracked squared norms as in the
//      other kernels);
//   3. X <- X Q (and V <- V Q) on the matrix cores, stored straight to the
//      work arrays.
// The convergence counts of a step (pairs whose cosine exceeds the rotation
// threshold, and the larger early-exit threshold) are taken from the fresh G
// before any rotation; every pair of the slice is a cross pair of exactly one
// step per sweep, and the pairs inside a block are counted at the sweep's
// first step, where they are rotated as well.  A step with nothing to rotate
// leaves its blocks as they are (no update and no store).
// ---------------------------------------------------------------------------
constexpr int kGramB = kGramBlock;         // columns per block
constexpr int kGramC = 2 * kGramB;         // columns per block pair
constexpr int kGramThreads = 256;          // four wavefronts
constexpr int kGramLd = kGramC + 1;        // leading dimension of G, K and Q in LDS (doubles)
constexpr int kGramRowsMax = kMaxRows / 64; // rows per lane when a wavefront loads one column
constexpr int kGramPM = kGramC * kGramLd;   // one 32 x 32 matrix with leading dimension 33

typedef float gram_f16v __attribute__((ext_vector_type(16)));
typedef double gram_d4v __attribute__((ext_vector_type(4)));
typedef __bf16 gram_bf8 __attribute__((ext_vector_type(8)));

// Padded rows of a block-pair column in LDS: m rounded up to 64, plus 4
// (FP32: a column starts 16-byte aligned, and the 16-byte operand reads of
// eight consecutive columns fall in distinct bank groups) or 1 (FP64: the
// 8-byte reads of 16 consecutive columns at one row fall in distinct banks).
__host__ __device__ inline int gram_ldx(int m, int es) { return (m + 63) / 64 * 64 + (es == 4 ? 4 : 1); }

// LDS bytes of the block-Gram kernel: the block pair, then G/K and Q (FP64,
// ld 33), then the tracked squared norms.
__host__ __device__ inline int gram_lds_bytes(int m, int es) {
    return kGramC * gram_ldx(m, es) * es + 2 * kGramPM * 8 + kGramC * 8;
}

// Global column of local column c (0..31) of the pair (BI, BJ).
__device__ __forceinline__ int gram_col(int c, int BI, int BJ) {
    return c < kGramB ? BI * kGramB + c : BJ * kGramB + (c - kGramB);
}

// One 16 x 16 tile (ti, tj) of G = X^T X of the block pair (rows [0, rows),
// LDS column-major with ld ldx) on the matrix cores, written to Kd (FP64,
// column-major, ld kGramLd).  mode 0: FP64 products; 1: FP32; 2: BF16 hi + lo
// (hi*hi + hi*lo + lo*hi, the lo*lo term dropped).  rows is a multiple of 32.
typedef float gram_f4v __attribute__((ext_vector_type(4)));
template <typename T>
__device__ void gram_tile(const T* __restrict__ Xs, int ldx, int rows, int mode, int ti, int tj,
                          double* __restrict__ Kd) {
    const int lane = threadIdx.x & 63, c16 = lane & 15, kq = lane >> 4;
    const T* xa = Xs + (int64_t)(16 * ti + c16) * ldx;
    const T* xb = Xs + (int64_t)(16 * tj + c16) * ldx;
    // four independent accumulators (K steps taken round robin) keep the
    // matrix-core pipeline full; they are added in a fixed order at the end
    if (mode == 0) {
        gram_d4v a0 = {0.0, 0.0, 0.0, 0.0}, a1 = a0, a2 = a0, a3 = a0;
        for (int k0 = 0; k0 < rows; k0 += 16) {
            a0 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)xa[k0 + kq], (double)xb[k0 + kq], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)xa[k0 + 4 + kq], (double)xb[k0 + 4 + kq], a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)xa[k0 + 8 + kq], (double)xb[k0 + 8 + kq], a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f64_16x16x4f64((double)xa[k0 + 12 + kq], (double)xb[k0 + 12 + kq], a3, 0, 0, 0);
        }
        // element v: row kq + 4 v, column c16
#pragma unroll
        for (int v = 0; v < 4; ++v)
            Kd[(16 * tj + c16) * kGramLd + 16 * ti + kq + 4 * v] = (a0[v] + a1[v]) + (a2[v] + a3[v]);
        return;
    }
    gram_f4v a0 = {0.f, 0.f, 0.f, 0.f}, a1 = a0, a2 = a0, a3 = a0;
    if (mode == 1) {
        for (int k0 = 0; k0 < rows; k0 += 16) {
            a0 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)xa[k0 + kq], (float)xb[k0 + kq], a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)xa[k0 + 4 + kq], (float)xb[k0 + 4 + kq], a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)xa[k0 + 8 + kq], (float)xb[k0 + 8 + kq], a2, 0, 0, 0);
            a3 = __builtin_amdgcn_mfma_f32_16x16x4f32((float)xa[k0 + 12 + kq], (float)xb[k0 + 12 + kq], a3, 0, 0, 0);
        }
    } else {
        // hi*hi, hi*lo and lo*hi in three accumulators
        for (int k0 = 0; k0 < rows; k0 += 32) {
            gram_bf8 ah, al, bh, bl;
            // eight consecutive rows of each column as two 16-byte reads
            float xr[8], yr[8];
            if constexpr (sizeof(T) == 4) {
                const float4* pa = (const float4*)(xa + k0 + 8 * kq);
                const float4* pb = (const float4*)(xb + k0 + 8 * kq);
                const float4 x0 = pa[0], x1 = pa[1], y0 = pb[0], y1 = pb[1];
                xr[0] = x0.x; xr[1] = x0.y; xr[2] = x0.z; xr[3] = x0.w;
                xr[4] = x1.x; xr[5] = x1.y; xr[6] = x1.z; xr[7] = x1.w;
                yr[0] = y0.x; yr[1] = y0.y; yr[2] = y0.z; yr[3] = y0.w;
                yr[4] = y1.x; yr[5] = y1.y; yr[6] = y1.z; yr[7] = y1.w;
            } else {
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    xr[e] = (float)xa[k0 + 8 * kq + e];
                    yr[e] = (float)xb[k0 + 8 * kq + e];
                }
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const float x = xr[e], y = yr[e];
                const __bf16 hx = (__bf16)x, hy = (__bf16)y;
                ah[e] = hx;
                al[e] = (__bf16)(x - (float)hx);
                bh[e] = hy;
                bl[e] = (__bf16)(y - (float)hy);
            }
            a0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, a0, 0, 0, 0);
            a1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, a1, 0, 0, 0);
            a2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, a2, 0, 0, 0);
        }
    }
    // element v: row 4 kq + v, column c16
#pragma unroll
    for (int v = 0; v < 4; ++v)
        Kd[(16 * tj + c16) * kGramLd + 16 * ti + 4 * kq + v] =
            ((double)a0[v] + (double)a1[v]) + ((double)a2[v] + (double)a3[v]);
}

// X_new = X Q for the block pair (rows [0, m)), written to the columns of the
// work array W (column gc(i) at W + gc ld); src is X in LDS (ld ldx), or,
// when from_global, the columns of W itself (rows < m read with L1-bypassing
// loads; used for V).  Computed transposed, X_new^T = Q^T X^T, so that the 32
// (FP32) or 16 (FP64) lanes of an output row of the matrix-core product walk
// down one column of X_new (contiguous stores).  f64: FP64 products (FP32
// data converted exactly, result rounded once).
template <typename T>
__device__ void gram_apply(const T* __restrict__ Xs, int ldx, bool from_global, T* __restrict__ W, int64_t ld,
                           int m, int BI, int BJ, int p, const double* __restrict__ Qd, bool f64) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    auto xval = [&](int k, int r) -> T {
        if (r >= m) return (T)0;
        if (!from_global) return Xs[(int64_t)k * ldx + r];
        const int gk = gram_col(k, BI, BJ);
        return gk < p ? ld_team(W + (int64_t)gk * ld + r) : (T)0;
    };
    if (sizeof(T) == 8 || f64) {
        // 16-row tiles, both 16-column halves of the output by the same
        // wavefront (its reads of a row tile all precede its stores to it)
        const int tj_n = (m + 15) / 16;
        for (int tj = wave; tj < tj_n; tj += 4) {
            const int j0 = tj * 16, r = j0 + (lane & 15);
            gram_d4v acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
            // A = Q^T tile: A[i][k] = Q[k][16 ti + i];  B[k][j] = X[j0 + j][k]
            double b[kGramC / 4];
#pragma unroll
            for (int q = 0; q < kGramC / 4; ++q) b[q] = (double)xval(4 * q + (lane >> 4), r);
#pragma unroll
            for (int q = 0; q < kGramC / 4; q += 2) {
                const int k = 4 * q + (lane >> 4);
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(Qd[(lane & 15) * kGramLd + k], b[q], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(Qd[(16 + (lane & 15)) * kGramLd + k], b[q], acc1, 0, 0, 0);
                acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(Qd[(lane & 15) * kGramLd + k + 4], b[q + 1], acc2, 0, 0, 0);
                acc3 = __builtin_amdgcn_mfma_f64_16x16x4f64(Qd[(16 + (lane & 15)) * kGramLd + k + 4], b[q + 1], acc3, 0,
                                                            0, 0);
            }
            acc0 += acc2;
            acc1 += acc3;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int i = (lane >> 4) + 4 * v;
                const int g0 = gram_col(i, BI, BJ), g1 = gram_col(16 + i, BI, BJ);
                if (r < m && g0 < p) W[(int64_t)g0 * ld + r] = (T)acc0[v];
                if (r < m && g1 < p) W[(int64_t)g1 * ld + r] = (T)acc1[v];
            }
        }
        return;
    }
    // FP32: 32 x 32 tiles over the rows; the Q^T operand is the same for every tile
    float qa[kGramC / 2];
#pragma unroll
    for (int s = 0; s < kGramC / 2; ++s) qa[s] = (float)Qd[(lane & 31) * kGramLd + 2 * s + (lane >> 5)];
    // two 32-row tiles per wavefront at a time (independent accumulators); all
    // of a tile's B operands are read before its products
    const int tj_n = (m + 31) / 32;
    for (int tj = wave; tj < tj_n; tj += 8) {
        const int ra = tj * 32 + (lane & 31), rb = ra + 128;
        const bool two = tj + 4 < tj_n;
        float ba[kGramC / 2], bb[kGramC / 2];
#pragma unroll
        for (int s = 0; s < kGramC / 2; ++s) {
            ba[s] = (float)xval(2 * s + (lane >> 5), ra);
            bb[s] = two ? (float)xval(2 * s + (lane >> 5), rb) : 0.0f;
        }
        gram_f16v acc = {}, acc2 = {}, acc3 = {}, acc4 = {};
#pragma unroll
        for (int s = 0; s < kGramC / 2; s += 2) {
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[s], ba[s], acc, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[s + 1], ba[s + 1], acc3, 0, 0, 0);
            if (two) {
                acc2 = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[s], bb[s], acc2, 0, 0, 0);
                acc4 = __builtin_amdgcn_mfma_f32_32x32x2f32(qa[s + 1], bb[s + 1], acc4, 0, 0, 0);
            }
        }
        acc += acc3;
        acc2 += acc4;
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int i = 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3), gi = gram_col(i, BI, BJ);
            if (ra < m && gi < p) W[(int64_t)gi * ld + ra] = (T)acc[v];
            if (two && rb < m && gi < p) W[(int64_t)gi * ld + rb] = (T)acc2[v];
        }
    }
}

// Sum of one int per thread over the workgroup's four wavefronts (every
// thread gets it): wavefront sums by lane swaps, then four LDS words.
__device__ __forceinline__ int block_sum_waves(int v, int* s_w4) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    __syncthreads();  // earlier readers of s_w4 are done
    if ((threadIdx.x & 63) == 0) s_w4[threadIdx.x >> 6] = v;
    __syncthreads();
    return s_w4[0] + s_w4[1] + s_w4[2] + s_w4[3];
}

// One slice by one team, block-Gram steps.  Returns false if a wait timed out.
template <typename T, bool WV>
__device__ bool gram_task(const JacobiJob& J, int k, int rank, TeamState& ts, int max_sweeps, unsigned char* lds,
                          int* s_w4, int* s_flag) {
    const int m = J.m, p = J.p, nb = J.nb;
    const int ldx = gram_ldx(m, (int)sizeof(T));
    const int mp = (m + 63) / 64 * 64;
    T* Xs = (T*)lds;
    double* Kd = (double*)(lds + (size_t)kGramC * ldx * sizeof(T));
    double* Qd = Kd + kGramPM;
    double* nrm = Qd + kGramPM;
    const int tid = threadIdx.x, wave = tid >> 6;
    const int grp = tid >> 4, gl = tid & 15;  // inner phase: 16 lane groups of 16
    const double tol = J.tol;
    const bool refine = J.refine64 != 0;
    int sweeps = -1, executed = 0;
    int* rot_g = J.rot + (int64_t)k * kRotStride;
    T* Ag = (T*)J.A + (int64_t)k * m * p;
    T* Vg = WV ? (T*)J.V + (int64_t)k * p * p : nullptr;
    for (int sw = 0; sw < max_sweeps + (refine ? 1 : 0); ++sw) {
        const bool f64 = refine && sw == max_sweeps;
        const double tl = f64 ? (double)m * Unit<double>::v : tol;
        const int mode = (sizeof(T) == 8 || f64) ? 0 : (refine ? 2 : 1);
        int rot = 0, big = 0;
        ++executed;
        for (int s = 0; s < nb - 1; ++s) {
            const bool last = (s == nb - 2);
            for (int q = rank; q < nb / 2; q += ts.W) {
                int BI, BJ;
                rr_pair(s, q, nb, BI, BJ);
                if (s > 0 && !team_wait_blocks(ts, BI, BJ, ts.steps, s_flag)) return false;
                const bool first = (sw == 0 && s == 0);
                // 1. the block pair into LDS (zero rows beyond m, zero columns beyond p)
                if (first && J.src_rs != 1) {
                    // transposed source: consecutive lanes take consecutive columns (contiguous
                    // in memory); thread t takes column t mod 32 and rows t / 32 + 8 q, eight
                    // loads in flight before their LDS stores
                    const int c = tid & 31, gc = gram_col(c, BI, BJ);
                    for (int q0 = 0; q0 < mp / 8; q0 += 8) {
                        T v[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) {
                            const int r = (tid >> 5) + 8 * (q0 + q);
                            v[q] = (r < m && gc < p) ? src_at<T>(J, k, r, gc) : (T)0;
                        }
#pragma unroll
                        for (int q = 0; q < 8; ++q) Xs[(int64_t)c * ldx + (tid >> 5) + 8 * (q0 + q)] = v[q];
                    }
                } else {
                    // wavefront w loads columns 8 w .. 8 w + 7, lane l rows l + 64 q: all of
                    // its loads are issued before its LDS stores
                    const int lane = tid & 63, nq = mp / 64;
                    T v[8][kGramRowsMax];
#pragma unroll
                    for (int cc = 0; cc < 8; ++cc) {
                        const int gc = gram_col(8 * wave + cc, BI, BJ);
#pragma unroll
                        for (int q = 0; q < kGramRowsMax; ++q) {
                            const int r = lane + 64 * q;
                            T x = (T)0;
                            if (q < nq && r < m && gc < p)
                                x = first ? src_at<T>(J, k, r, gc) : ld_team(Ag + (int64_t)gc * m + r);
                            v[cc][q] = x;
                        }
                    }
#pragma unroll
                    for (int cc = 0; cc < 8; ++cc) {
#pragma unroll
                        for (int q = 0; q < kGramRowsMax; ++q)
                            if (q < nq) Xs[(int64_t)(8 * wave + cc) * ldx + lane + 64 * q] = v[cc][q];
                    }
                }
                __syncthreads();
                // 2. G = X^T X: wavefront w computes tile (w / 2, w mod 2) over all rows
                gram_tile<T>(Xs, ldx, mp, mode, wave >> 1, wave & 1, Kd);
                for (int e = tid; e < kGramC * kGramC; e += kGramThreads) {
                    const int c = e >> 5, r = e & 31;
                    Qd[c * kGramLd + r] = r == c ? 1.0 : 0.0;
                }
                __syncthreads();
                if (tid < kGramC) nrm[tid] = Kd[tid * kGramLd + tid];
                const int cj = tid & 31;
                // convergence counts of this step's pairs (i < j) from the fresh G
                int cnt = 0;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int ri = (tid >> 5) + 8 * q;
                    if (cj <= ri) continue;
                    const bool cross = (ri < kGramB) != (cj < kGramB);
                    if (!cross && s != 0) continue;
                    if (gram_col(ri, BI, BJ) >= p || gram_col(cj, BI, BJ) >= p) continue;
                    const double g = Kd[cj * kGramLd + ri], ab = Kd[ri * kGramLd + ri] * Kd[cj * kGramLd + cj];
                    cnt += !(g * g <= (tl * tl) * ab);           // would rotate (count in the low half)
                    cnt += !(g * g <= J.skip2 * ab) ? 65536 : 0;  // large cosine (high half)
                }
                cnt = block_sum_waves(cnt, s_w4);
                const int nrot = cnt & 0xFFFF, nbig = cnt >> 16;
                rot += (tid == 0) ? nrot : 0;
                big += (tid == 0) ? nbig : 0;
                // 3. the step's rotations on (Q, K): 16 lane groups, two rows of 32 per lane
                int moved = 0;
                if (nrot > 0 && s != 0) {
                    // cross rounds: group g = 4 w + u keeps I column g (its Q and K rows) in
                    // registers; the J columns form four sub-blocks of four, and in super-round
                    // R wavefront w owns sub-block (w + R) mod 4, whose columns pass among its
                    // four groups (group u meets column (u + v) mod 4 in sub-round v).  LDS
                    // accesses of one wavefront complete in program order, so only the
                    // super-rounds end at a workgroup barrier.
                    const int u = grp & 3, i = grp;
                    double* qi = Qd + i * kGramLd;
                    double* ki = Kd + i * kGramLd;
                    double q0 = qi[gl], q1 = qi[gl + 16], k0 = ki[gl], k1 = ki[gl + 16];
                    double a = nrm[i];
                    for (int R = 0; R < 4; ++R) {
                        const int sb = (wave + R) & 3;
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int j = kGramB + 4 * sb + ((u + v) & 3);
                            double* qj = Qd + j * kGramLd;
                            double* kj = Kd + j * kGramLd;
                            const double r0_ = qj[gl], r1 = qj[gl + 16], l0 = kj[gl], l1 = kj[gl + 16];
                            const double b = nrm[j];
                            const double g = group_sum<16>(fma(q0, l0, q1 * l1));
                            double c, sn, t;
                            if (rotation(a, b, g, tl, c, sn, t)) {
                                qj[gl] = sn * q0 + c * r0_;
                                qj[gl + 16] = sn * q1 + c * r1;
                                kj[gl] = sn * k0 + c * l0;
                                kj[gl + 16] = sn * k1 + c * l1;
                                q0 = c * q0 - sn * r0_;
                                q1 = c * q1 - sn * r1;
                                k0 = c * k0 - sn * l0;
                                k1 = c * k1 - sn * l1;
                                if (gl == 0) nrm[j] = b + t * g;
                                a -= t * g;
                                moved = 1;
                            }
                            // keeps the next sub-round's LDS reads below this one's writes
                            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                        }
                        __syncthreads();
                    }
                    qi[gl] = q0;
                    qi[gl + 16] = q1;
                    __syncthreads();
                } else if (nrot > 0) {
                    // the sweep's first step: all pairs of the 32 columns, both in LDS
                    for (int r = 0; r < kGramC - 1; ++r) {
                        int i, j;
                        rr_pair(r, grp, kGramC, i, j);
                        double* qi = Qd + i * kGramLd;
                        double* qj = Qd + j * kGramLd;
                        double* ki = Kd + i * kGramLd;
                        double* kj = Kd + j * kGramLd;
                        const double q0 = qi[gl], q1 = qi[gl + 16], r0_ = qj[gl], r1 = qj[gl + 16];
                        const double k0 = ki[gl], k1 = ki[gl + 16], l0 = kj[gl], l1 = kj[gl + 16];
                        const double a = nrm[i], b = nrm[j];
                        const double g = group_sum<16>(fma(q0, l0, q1 * l1));
                        double c, sn, t;
                        if (rotation(a, b, g, tl, c, sn, t)) {
                            qi[gl] = c * q0 - sn * r0_; qj[gl] = sn * q0 + c * r0_;
                            qi[gl + 16] = c * q1 - sn * r1; qj[gl + 16] = sn * q1 + c * r1;
                            ki[gl] = c * k0 - sn * l0; kj[gl] = sn * k0 + c * l0;
                            ki[gl + 16] = c * k1 - sn * l1; kj[gl + 16] = sn * k1 + c * l1;
                            if (gl == 0) {
                                nrm[i] = a - t * g;
                                nrm[j] = b + t * g;
                            }
                            moved = 1;
                        }
                        __syncthreads();
                    }
                }
                moved = block_sum_waves(moved, s_w4);
                // 4. X <- X Q and V <- V Q straight to the work arrays; a first step that
                // rotated nothing still copies the source into A
                if (moved) {
                    gram_apply<T>(Xs, ldx, false, Ag, m, m, BI, BJ, p, Qd, f64);
                    if (WV) gram_apply<T>(Xs, ldx, true, Vg, p, p, BI, BJ, p, Qd, f64);
                } else if (first) {
                    for (int e = tid; e < kGramC * m; e += kGramThreads) {
                        const int c = e / m, r = e - c * m, gc = gram_col(c, BI, BJ);
                        if (gc < p) Ag[(int64_t)gc * m + r] = Xs[(int64_t)c * ldx + r];
                    }
                }
                if (!last) team_release_blocks(ts, BI, BJ, ts.steps + 1);
                else __syncthreads();
            }
            ts.steps += 1;
            if (last) {
                if (tid == 0 && rot) atomicAdd(rot_g + sw, rot);
                if (tid == 0 && big) atomicAdd(rot_g + kMaxSweeps + sw, big);
                if (!team_barrier(ts, s_flag)) return false;
            }
        }
        if (f64) break;
        const int total = __hip_atomic_load(rot_g + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int large = __hip_atomic_load(rot_g + kMaxSweeps + sw, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (total == 0 || large == 0) {
            sweeps = sw + 1;
            if (!refine) break;
            sw = max_sweeps - 1;
        }
    }
    if (tid == 0 && rank == 0) record_slice(J, k, sweeps, executed, ts.ctrl);
    return true;
}

template <typename T, bool WV>
__global__ __launch_bounds__(kGramThreads) void k_jacobi_gram(JacobiJob J1, int ntasks, TeamSched sched,
                                                             int max_sweeps, Ctrl* ctrl, int spin_limit) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    __shared__ int s_w4[4], s_flag, s_team, s_rank, s_nteams;
    const int W = sched.W;
    int* ctl = sched.ctl;
    if (threadIdx.x == 0) {
        const int x = xcc_id();
        const int slot = __hip_atomic_fetch_add(ctl + x, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(ctl + 16, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int it = 0;
        bool ok = true;
        while (__hip_atomic_load(ctl + 16, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < (int)gridDim.x) {
            if (++it > spin_limit) {
                atomicOr(&ctrl->status, kStTimeout);
                ok = false;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        int before = 0, total = 0;
        for (int xx = 0; xx < 16; ++xx) {
            const int full = __hip_atomic_load(ctl + xx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) / W;
            if (xx < x) before += full;
            total += full;
        }
        const int local = slot / W;
        const int full_here = __hip_atomic_load(ctl + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) / W;
        s_team = (ok && local < full_here) ? before + local : -1;
        s_rank = slot % W;
        s_nteams = total;
        if (ok && total == 0 && blockIdx.x == 0) atomicOr(&ctrl->status, kStTimeout);
    }
    __syncthreads();
    const int team = s_team, rank = s_rank, nteams = s_nteams;
    if (team < 0) return;
    TeamState ts{ctl + 32 + team * W, 0, W, spin_limit, ctrl, rank, ctl + 32 + gridDim.x + team * J1.nb, 0};
    for (int t = team; t < ntasks; t += nteams)
        if (!gram_task<T, WV>(J1, t, rank, ts, max_sweeps, smem_raw, s_w4, &s_flag)) return;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
static int elem_size(int prec) { return prec == 0 ? 8 : 4; }

int jacobi_geometry_g(int m, int p, int G, int* R, int* ldv) {
    if (G != 16 && G != 32 && G != 64) return -1;
    int r = (m + G - 1) / G;
    r = (r + 3) / 4 * 4;
    if (r < 4) r = 4;
    if (r > 16) return -1;
    *R = r;
    *ldv = ((p + G - 1) / G) * G;
    return 0;
}

void jacobi_geometry(int m, int p, int* G, int* R, int* ldv) {
    *G = m <= 256 ? 16 : 32;
    (void)jacobi_geometry_g(m, p, *G, R, ldv);
}

int jacobi_resident_lds_bytes(int prec, int m, int p, int G, int with_v) {
    int R, ldv;
    if (jacobi_geometry_g(m, p, G, &R, &ldv)) return 1 << 30;
    const int pp = p + (p & 1);
    const int64_t elems = (int64_t)pp * (R * G + kLdsPad) + (with_v ? (int64_t)pp * ldv : 0);
    return (int)(elems * elem_size(prec));
}

int jacobi_team_lds_bytes(int prec, int m, int p, int G, int b, int with_v) {
    int R, ldv;
    if (jacobi_geometry_g(m, p, G, &R, &ldv)) return 1 << 30;
    // two blocks of b columns; with V each column holds R G rows of V below its R G rows of A
    const int64_t elems = (int64_t)2 * b * ((with_v ? 2 : 1) * R * G + kLdsPad);
    return (int)(elems * elem_size(prec));
}

template <typename T, bool WV, int K>
static const void* team_fn_rg(int R, int G) {
    if (G == 16) {
        switch (R) {
            case 4: return (const void*)k_jacobi_team<T, WV, 4, 16, K>;
            case 8: return (const void*)k_jacobi_team<T, WV, 8, 16, K>;
            case 12: return (const void*)k_jacobi_team<T, WV, 12, 16, K>;
            default: return (const void*)k_jacobi_team<T, WV, 16, 16, K>;
        }
    }
    if (G == 64) {
        if constexpr (K == 1) {
            switch (R) {
                case 4: return (const void*)k_jacobi_team<T, WV, 4, 64, 1>;
                case 8: return (const void*)k_jacobi_team<T, WV, 8, 64, 1>;
                case 12: return (const void*)k_jacobi_team<T, WV, 12, 64, 1>;
                default: return (const void*)k_jacobi_team<T, WV, 16, 64, 1>;
            }
        }
        return nullptr;  // two columns per group: 16- and 32-lane groups only
    }
    switch (R) {
        case 4: return (const void*)k_jacobi_team<T, WV, 4, 32, K>;
        case 8: return (const void*)k_jacobi_team<T, WV, 8, 32, K>;
        case 12: return (const void*)k_jacobi_team<T, WV, 12, 32, K>;
        default: return (const void*)k_jacobi_team<T, WV, 16, 32, K>;
    }
}
// K = 2 (two columns per lane group) exists without V only
static const void* team_fn(int prec, int with_v, int R, int G, int K) {
    if (K == 2)
        return prec == 0 ? team_fn_rg<double, false, 2>(R, G) : team_fn_rg<float, false, 2>(R, G);
    return prec == 0 ? (with_v ? team_fn_rg<double, true, 1>(R, G) : team_fn_rg<double, false, 1>(R, G))
                     : (with_v ? team_fn_rg<float, true, 1>(R, G) : team_fn_rg<float, false, 1>(R, G));
}
template <typename T, bool WV>
static const void* res_fn() { return (const void*)k_jacobi_resident<T, WV>; }

hipError_t launch_jacobi_resident(int prec, const JacobiJob& job1, const JacobiJob* jobs_dev, const int* task_job,
                                  const int* task_slice, int ntasks, int max_sweeps, Ctrl* ctrl, int lds_bytes,
                                  int threads, int with_v, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    const void* f = prec == 0 ? (with_v ? res_fn<double, true>() : res_fn<double, false>())
                              : (with_v ? res_fn<float, true>() : res_fn<float, false>());
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
    JacobiJob j1 = job1;
    void* args[] = {(void*)&j1, (void*)&jobs_dev, (void*)&task_job, (void*)&task_slice,
                    (void*)&ntasks, (void*)&max_sweeps, (void*)&ctrl};
    return hipLaunchKernel(f, dim3(ntasks), dim3(threads), args, (size_t)lds_bytes, s);
}

hipError_t launch_jacobi_team(int prec, const JacobiJob& job, int ntasks, const TeamSched& ts_in, int max_sweeps,
                              Ctrl* ctrl, int lds_bytes, int threads, int with_v, int spin_limit, int R, int G, int K,
                              int coop, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    if (K == 2 && with_v) return hipErrorInvalidValue;
    const void* f = team_fn(prec, with_v, R, G, K);
    if (!f) return hipErrorInvalidValue;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
    TeamSched ts = ts_in;
    JacobiJob j1 = job;
    void* args[] = {(void*)&j1, (void*)&ntasks, (void*)&ts, (void*)&max_sweeps, (void*)&ctrl, (void*)&spin_limit};
    dim3 grid(ts.nwg), block(threads);
    if (coop) return hipLaunchCooperativeKernel(f, grid, block, args, (unsigned)lds_bytes, s);
    // plain launch (inside stream capture): the grid fits the device, and the
    // bounded team waits turn a non-resident team into an error, not a hang
    return hipLaunchKernel(f, grid, block, args, (size_t)lds_bytes, s);
}

template <typename T, bool WV>
static const void* batched_fn_t(int R, int G) {
    if (G == 16) {
        switch (R) {
            case 4: return (const void*)k_jacobi_batched<T, 4, 16, WV>;
            case 8: return (const void*)k_jacobi_batched<T, 8, 16, WV>;
            case 12: return (const void*)k_jacobi_batched<T, 12, 16, WV>;
            default: return (const void*)k_jacobi_batched<T, 16, 16, WV>;
        }
    }
    switch (R) {
        case 4: return (const void*)k_jacobi_batched<T, 4, 32, WV>;
        case 8: return (const void*)k_jacobi_batched<T, 8, 32, WV>;
        case 12: return (const void*)k_jacobi_batched<T, 12, 32, WV>;
        default: return (const void*)k_jacobi_batched<T, 16, 32, WV>;
    }
}

hipError_t launch_jacobi_batched(int prec, int R, int G, int with_v, const JacobiJob* jobs_dev, const int* task_job,
                                 const int* task_slice, int ntasks, int* queue, int max_sweeps, Ctrl* ctrl,
                                 int lds_bytes, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    const void* f = prec == 0 ? (with_v ? batched_fn_t<double, true>(R, G) : batched_fn_t<double, false>(R, G))
                              : (with_v ? batched_fn_t<float, true>(R, G) : batched_fn_t<float, false>(R, G));
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) return e;
    int per_cu = 0, dev = 0, cus = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, kTeamMaxThreads, lds_bytes);
    if (e != hipSuccess) return e;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int grid = std::max(1, std::min(ntasks, std::max(1, per_cu) * cus));
    void* args[] = {(void*)&jobs_dev, (void*)&task_job, (void*)&task_slice, (void*)&ntasks,
                    (void*)&queue,    (void*)&max_sweeps, (void*)&ctrl};
    return hipLaunchKernel(f, dim3(grid), dim3(kTeamMaxThreads), args, (size_t)lds_bytes, s);
}


// ---- block-Gram kernel ---------------------------------------------------------
__global__ void k_identity(void* V, int p, int64_t total, int es) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t o = e % ((int64_t)p * p);
        const double v = (o % p) == (o / p) ? 1.0 : 0.0;
        if (es == 8) ((double*)V)[e] = v;
        else ((float*)V)[e] = (float)v;
    }
}

static const void* gram_fn(int prec, int with_v) {
    return prec == 0 ? (with_v ? (const void*)k_jacobi_gram<double, true> : (const void*)k_jacobi_gram<double, false>)
                     : (with_v ? (const void*)k_jacobi_gram<float, true> : (const void*)k_jacobi_gram<float, false>);
}

int jacobi_gram_lds_bytes(int prec, int m) { return gram_lds_bytes(m, elem_size(prec)); }

int jacobi_gram_max_resident(int prec, int m, int with_v) {
    const void* f = gram_fn(prec, with_v);
    const int lds = jacobi_gram_lds_bytes(prec, m);
    if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kGramThreads, lds) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, f) == hipSuccess && fa.numRegs > 0) {
        // one wavefront per SIMD per workgroup: at most 512 / VGPRs workgroups per CU
        const int vg = (fa.numRegs + 7) / 8 * 8;
        nb = std::min(nb, std::min(8, 512 / vg));
    } else {
        (void)hipGetLastError();
        nb = std::min(nb, 1);
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return nb * cus;
}

hipError_t launch_jacobi_gram(int prec, const JacobiJob& job, int ntasks, const TeamSched& ts_in, int max_sweeps,
                              Ctrl* ctrl, int with_v, int spin_limit, int coop, hipStream_t s) {
    if (ntasks <= 0) return hipSuccess;
    if (job.b != kGramB) return hipErrorInvalidValue;
    if (with_v && !job.vinit) {
        // the kernel reads V from the work array: start it at the identity
        const int64_t total = (int64_t)job.p * job.p * ntasks;
        const unsigned blocks = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 4096));
        hipLaunchKernelGGL(k_identity, dim3(blocks), dim3(256), 0, s, job.V, job.p, total, elem_size(prec));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const void* f = gram_fn(prec, with_v);
    const int lds = jacobi_gram_lds_bytes(prec, job.m);
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
    TeamSched ts = ts_in;
    JacobiJob j1 = job;
    void* args[] = {(void*)&j1, (void*)&ntasks, (void*)&ts, (void*)&max_sweeps, (void*)&ctrl, (void*)&spin_limit};
    dim3 grid(ts.nwg), block(kGramThreads);
    if (coop) return hipLaunchCooperativeKernel(f, grid, block, args, (unsigned)lds, s);
    return hipLaunchKernel(f, grid, block, args, (size_t)lds, s);
}

int jacobi_team_max_resident(int prec, int lds_bytes, int threads, int with_v, int R, int G, int K) {
    int nb = 0;
    if (K == 2 && with_v) return 0;
    const void* f = team_fn(prec, with_v, R, G, K);
    if (!f) return 0;
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();  // do not leave a sticky error for the caller's runtime
        return 0;
    }
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, threads, lds_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    // Workgroups per CU by registers counted per SIMD: a workgroup of w
    // wavefronts puts up to ceil(w/4) of them on one of the CU's 4 SIMDs, and a
    // SIMD holds 512 / (VGPRs rounded to 8) wavefronts.  With 6 wavefronts of
    // 149 VGPRs the occupancy query allows 2 workgroups per CU (12 of 12
    // wavefronts), but only one fits the SIMDs, and a team whose members cannot
    // all be resident would wait until its bounded spin gives up.
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, f) == hipSuccess && fa.numRegs > 0) {
        const int vg = (fa.numRegs + 7) / 8 * 8;
        const int per_simd = std::min(8, 512 / vg);
        const int waves = (threads + kWave - 1) / kWave;
        nb = std::min(nb, per_simd / ((waves + 3) / 4));
    } else {
        (void)hipGetLastError();
        nb = std::min(nb, 1);
    }
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return nb * cus;
}

}  // namespace tsvd
