/*
 * Plain FP64 CPU oracle for cosine-transform t-SVD, t-SVT and TNN-C tensor
 * completion (Xu, Zhao, Ng, "A Fast Algorithm for Cosine Transform Based
 * Tensor Singular Value Decomposition", arXiv 1902.03070).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares
 * no code, header, table or helper with the GPU library, and the GPU library
 * never calls it.
 *
 * Conventions (all functions):
 *   - A real tensor X of size n1 x n2 x n3 is stored column-major with frontal
 *     slices contiguous: X(i,j,k) lives at X[i + n1*j + n1*n2*k], 0-based.
 *   - Matrices are column-major: M(r,c) at M[r + ld*c].
 *   - C is the orthonormal DCT-II matrix of size n, stored row-major
 *     C[k*n + t] (row k = frequency, column t = tube position).
 *   - Everything is double precision; there is no blocking, no fusion and no
 *     reordering beyond the textbook definitions cited at each function.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define X3(i, j, k, n1, n2) ((int64_t)(i) + (int64_t)(n1) * ((int64_t)(j) + (int64_t)(n2) * (int64_t)(k)))

/* ------------------------------------------------------------------------- */
/* Host threads.  Work that is independent by construction (the frontal      */
/* slices of the transform domain, the lateral index of the tube transforms) */
/* may be split over or_set_threads(T) POSIX threads in contiguous chunks.   */
/* Each item's arithmetic is exactly the single-threaded one, so results are */
/* bitwise identical for every T.  Default: 1 thread.                         */
/* ------------------------------------------------------------------------- */
static int g_threads = 1;
void or_set_threads(int t) { g_threads = t < 1 ? 1 : (t > 256 ? 256 : t); }
int or_get_threads(void) { return g_threads; }

typedef void (*range_fn)(void* ctx, int64_t begin, int64_t end);
struct range_job { range_fn fn; void* ctx; int64_t begin, end; };
static void* range_run(void* a) {
    struct range_job* j = (struct range_job*)a;
    j->fn(j->ctx, j->begin, j->end);
    return NULL;
}
/* fn(ctx, b, e) over [0, n) split into min(T, n) contiguous chunks. */
static void parallel_for(int64_t n, range_fn fn, void* ctx) {
    int T = g_threads;
    if (T > n) T = (int)n;
    if (T <= 1) { if (n > 0) fn(ctx, 0, n); return; }
    pthread_t th[256];
    struct range_job jobs[256];
    for (int t = 0; t < T; ++t) {
        jobs[t].fn = fn; jobs[t].ctx = ctx;
        jobs[t].begin = n * t / T; jobs[t].end = n * (t + 1) / T;
    }
    for (int t = 1; t < T; ++t) pthread_create(&th[t], NULL, range_run, &jobs[t]);
    range_run(&jobs[0]);
    for (int t = 1; t < T; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------- */
/* Section 3: the cosine transform along tubes.                              */
/* The paper writes dct(X,[],3), MATLAB's orthonormal DCT-II, and never       */
/* prints the matrix; this is the standard orthonormal DCT-II matrix:         */
/*   C[k][t] = s_k cos(pi (2t+1) k / (2n)),  s_0 = sqrt(1/n), s_k = sqrt(2/n). */
/* The integer (2t+1) k is reduced modulo 4n (the cosine's period in these    */
/* units) before the cosine, so the argument stays below 2 pi and is rounded  */
/* once, whatever n.                                                          */
/* ------------------------------------------------------------------------- */
void or_dct_matrix(int n, double* C) {
    const double pi = acos(-1.0);
    for (int k = 0; k < n; ++k) {
        double s = (k == 0) ? sqrt(1.0 / n) : sqrt(2.0 / n);
        for (int t = 0; t < n; ++t) {
            const int64_t q = ((2 * (int64_t)t + 1) * k) % (4 * (int64_t)n);
            C[(int64_t)k * n + t] = s * cos(pi * (double)q / (2.0 * n));
        }
    }
}

/* Tube transform with a given n3 x n3 matrix M (row-major):
 *   out(i,j,k) = sum_t M[k][t] in(i,j,t)   (trans = 0), or
 *   out(i,j,t) = sum_k M[k][t] in(i,j,k)   (trans = 1, the product with M^T). */
struct tube_ctx { int64_t n1, n2, n3; const double* M; const double* in; double* out; int trans; };
static void tube_range(void* a, int64_t j0, int64_t j1) {
    const struct tube_ctx* c = (const struct tube_ctx*)a;
    const int64_t n1 = c->n1, n2 = c->n2, n3 = c->n3;
    for (int64_t j = j0; j < j1; ++j)
        for (int64_t i = 0; i < n1; ++i)
            for (int64_t k = 0; k < n3; ++k) {
                double acc = 0.0;
                for (int64_t t = 0; t < n3; ++t)
                    acc += (c->trans ? c->M[t * n3 + k] : c->M[k * n3 + t]) * c->in[X3(i, j, t, n1, n2)];
                c->out[X3(i, j, k, n1, n2)] = acc;
            }
}
static void tube_apply(int64_t n1, int64_t n2, int64_t n3, const double* M, int trans, const double* in, double* out) {
    struct tube_ctx c = {n1, n2, n3, M, in, out, trans};
    parallel_for(n2, tube_range, &c);
}

/* Xbar(:,:,k) = sum_t C[k][t] X(:,:,t)   (Section 3, Xbar = dct(X,[],3)). */
void or_dct_tubes(int64_t n1, int64_t n2, int64_t n3, const double* X, double* Xbar) {
    double* C = (double*)malloc(sizeof(double) * n3 * n3);
    or_dct_matrix((int)n3, C);
    tube_apply(n1, n2, n3, C, 0, X, Xbar);
    free(C);
}

/* Inverse: X(:,:,t) = sum_k C[k][t] Xbar(:,:,k)  (C orthonormal, so C^{-1} = C^T). */
void or_idct_tubes(int64_t n1, int64_t n2, int64_t n3, const double* Xbar, double* X) {
    double* C = (double*)malloc(sizeof(double) * n3 * n3);
    or_dct_matrix((int)n3, C);
    tube_apply(n1, n2, n3, C, 1, Xbar, X);
    free(C);
}

/* ------------------------------------------------------------------------- */
/* Section 3: the split X = A + sigma(A), where sigma shifts the frontal      */
/* slices up by one and appends a zero slice.  Solving slice by slice from   */
/* the last one: A^(n3) = X^(n3), A^(k) = X^(k) - A^(k+1).                    */
/* ------------------------------------------------------------------------- */
void or_split_shift(int64_t n1, int64_t n2, int64_t n3, const double* X, double* A) {
    int64_t s = n1 * n2;
    for (int64_t k = n3 - 1; k >= 0; --k)
        for (int64_t e = 0; e < s; ++e) A[k * s + e] = (k == n3 - 1) ? X[k * s + e] : X[k * s + e] - A[(k + 1) * s + e];
}

/* Section 3, block Toeplitz bt(A): block (r,c) = A^(|r-c|+1) (1-based slices).
 * Output is (n1*n3) x (n2*n3), column-major, leading dimension n1*n3. */
void or_bt(int64_t n1, int64_t n2, int64_t n3, const double* A, double* M) {
    int64_t ld = n1 * n3, s = n1 * n2;
    for (int64_t bc = 0; bc < n3; ++bc)
        for (int64_t br = 0; br < n3; ++br) {
            int64_t k = br > bc ? br - bc : bc - br; /* 0-based slice index */
            for (int64_t j = 0; j < n2; ++j)
                for (int64_t i = 0; i < n1; ++i) M[(br * n1 + i) + ld * (bc * n2 + j)] = A[k * s + i + n1 * j];
        }
}

/* Section 3, block Hankel bh(A): first block row A^(2),...,A^(n3),O and
 * last block row O,A^(n3),...,A^(2).  With q = r+c+2 for the 0-based block
 * (r,c), the block is A^(q) (1-based) when q <= n3, O when q = n3+1, and the
 * reflected slice A^(2 n3 + 2 - q) beyond. */
void or_bh(int64_t n1, int64_t n2, int64_t n3, const double* A, double* M) {
    int64_t ld = n1 * n3, s = n1 * n2;
    for (int64_t bc = 0; bc < n3; ++bc)
        for (int64_t br = 0; br < n3; ++br) {
            int64_t q = br + bc + 2;        /* 1-based index along the anti-diagonal */
            int64_t k1;                      /* 1-based slice index, 0 = zero block */
            if (q <= n3) k1 = q;
            else if (q == n3 + 1) k1 = 0;
            else k1 = 2 * n3 + 2 - q;
            for (int64_t j = 0; j < n2; ++j)
                for (int64_t i = 0; i < n1; ++i)
                    M[(br * n1 + i) + ld * (bc * n2 + j)] = (k1 == 0) ? 0.0 : A[(k1 - 1) * s + i + n1 * j];
        }
}

/* Section 3: btph(A) = bt(A) + bh(A). */
void or_btph(int64_t n1, int64_t n2, int64_t n3, const double* A, double* M) {
    int64_t ld = n1 * n3, cols = n2 * n3;
    double* H = (double*)malloc(sizeof(double) * ld * cols);
    or_bt(n1, n2, n3, A, M);
    or_bh(n1, n2, n3, A, H);
    for (int64_t e = 0; e < ld * cols; ++e) M[e] += H[e];
    free(H);
}

/* Section 2, unfold: stack the frontal slices vertically into an
 * (n1*n3) x n2 column-major matrix; fold is its inverse. */
void or_unfold(int64_t n1, int64_t n2, int64_t n3, const double* X, double* U) {
    int64_t ld = n1 * n3;
    for (int64_t k = 0; k < n3; ++k)
        for (int64_t j = 0; j < n2; ++j)
            for (int64_t i = 0; i < n1; ++i) U[(k * n1 + i) + ld * j] = X[X3(i, j, k, n1, n2)];
}
void or_fold(int64_t n1, int64_t n2, int64_t n3, const double* U, double* X) {
    int64_t ld = n1 * n3;
    for (int64_t k = 0; k < n3; ++k)
        for (int64_t j = 0; j < n2; ++j)
            for (int64_t i = 0; i < n1; ++i) X[X3(i, j, k, n1, n2)] = U[(k * n1 + i) + ld * j];
}

/* Plain column-major matrix product C(m x n) = A(m x k) B(k x n). */
static void matmul(int64_t m, int64_t n, int64_t kk, const double* A, int64_t lda, const double* B, int64_t ldb,
                   double* C, int64_t ldc) {
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < m; ++r) {
            double acc = 0.0;
            for (int64_t t = 0; t < kk; ++t) acc += A[r + lda * t] * B[t + ldb * c];
            C[r + ldc * c] = acc;
        }
}

/* Definition (DCT-based t-product), the form built from the definition:
 * Z = fold(btph(A) unfold(Y)) with X = A + sigma(A).
 * X: n1 x n2 x n3, Y: n2 x n4 x n3, Z: n1 x n4 x n3. */
void or_btph_product(int64_t n1, int64_t n2, int64_t n4, int64_t n3, const double* X, const double* Y, double* Z) {
    double* A = (double*)malloc(sizeof(double) * n1 * n2 * n3);
    double* M = (double*)malloc(sizeof(double) * n1 * n3 * n2 * n3);
    double* UY = (double*)malloc(sizeof(double) * n2 * n3 * n4);
    double* UZ = (double*)malloc(sizeof(double) * n1 * n3 * n4);
    or_split_shift(n1, n2, n3, X, A);
    or_btph(n1, n2, n3, A, M);
    or_unfold(n2, n4, n3, Y, UY);
    matmul(n1 * n3, n4, n2 * n3, M, n1 * n3, UY, n2 * n3, UZ, n1 * n3);
    or_fold(n1, n4, n3, UZ, Z);
    free(A); free(M); free(UY); free(UZ);
}

/* Equation (tproduct dct), the transform-domain form used by Theorem 4,
 * TNN-C and Algorithm 1: Zbar^(k) = Xbar^(k) Ybar^(k), then Z = idct(Zbar). */
void or_tprod_dct(int64_t n1, int64_t n2, int64_t n4, int64_t n3, const double* X, const double* Y, double* Z) {
    double* Xb = (double*)malloc(sizeof(double) * n1 * n2 * n3);
    double* Yb = (double*)malloc(sizeof(double) * n2 * n4 * n3);
    double* Zb = (double*)malloc(sizeof(double) * n1 * n4 * n3);
    or_dct_tubes(n1, n2, n3, X, Xb);
    or_dct_tubes(n2, n4, n3, Y, Yb);
    for (int64_t k = 0; k < n3; ++k)
        matmul(n1, n4, n2, Xb + k * n1 * n2, n1, Yb + k * n2 * n4, n2, Zb + k * n1 * n4, n1);
    or_idct_tubes(n1, n4, n3, Zb, Z);
    free(Xb); free(Yb); free(Zb);
}

/* ------------------------------------------------------------------------- */
/* Thin SVD of one real matrix by the one-sided Jacobi method of Hestenes    */
/* (1958), as presented by Demmel and Veselic (1992) and Golub and Van Loan. */
/* The paper takes the SVD of each transformed frontal slice (Theorem 4 and  */
/* Algorithm 1) with a library routine and fixes no method; this is the     */
/* textbook cyclic-by-row one-sided Jacobi:                                  */
/*   for each pair i<j of columns of W: alpha=|w_i|^2, beta=|w_j|^2,          */
/*   gamma=w_i.w_j; if |gamma| > tol*sqrt(alpha*beta) rotate so that the two  */
/*   columns become orthogonal; stop after a sweep with no rotation.          */
/* A is m x n with leading dimension lda.  p = min(m,n).  Outputs:            */
/*   U: m x p, s: p (descending), V: n x p, all column-major; any may be NULL.*/
/* Signs: each (u_j, v_j) is flipped so that the entry of u_j of largest     */
/* magnitude (first one on ties) is positive.  A zero singular value gets a  */
/* u_j completed by Gram-Schmidt against e_1, e_2, ...                        */
/* Returns the number of sweeps, or -1 if max_sweeps was reached.             */
/* ------------------------------------------------------------------------- */
static int jacobi_tall(int64_t m, int64_t n, double* W, double* V, int max_sweeps, double tol) {
    /* W: m x n (m >= n), rotated in place; V: n x n, starts as the identity. */
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < n; ++r) V[r + n * c] = (r == c) ? 1.0 : 0.0;
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int64_t rotations = 0;
        for (int64_t i = 0; i < n - 1; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double* wi = W + m * i;
                double* wj = W + m * j;
                double alpha = 0.0, beta = 0.0, gamma = 0.0;
                for (int64_t r = 0; r < m; ++r) {
                    alpha += wi[r] * wi[r];
                    beta += wj[r] * wj[r];
                    gamma += wi[r] * wj[r];
                }
                if (gamma == 0.0 || fabs(gamma) <= tol * sqrt(alpha * beta)) continue;
                double zeta = (beta - alpha) / (2.0 * gamma);
                double sgn = (zeta >= 0.0) ? 1.0 : -1.0;
                double t = sgn / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t r = 0; r < m; ++r) {
                    double a = wi[r], b = wj[r];
                    wi[r] = c * a - s * b;
                    wj[r] = s * a + c * b;
                }
                double* vi = V + n * i;
                double* vj = V + n * j;
                for (int64_t r = 0; r < n; ++r) {
                    double a = vi[r], b = vj[r];
                    vi[r] = c * a - s * b;
                    vj[r] = s * a + c * b;
                }
                ++rotations;
            }
        if (rotations == 0) return sweep;
    }
    return -1;
}

/* Column c of Q (m rows, ld m) := a unit vector orthogonal to the columns
 * use[0..nuse): the standard basis vector e_i with the largest part outside
 * their span (1 - sum_q Q[i][q]^2; first i on ties), projected out twice
 * (Gram-Schmidt, one column at a time) and normalized. */
static void complement_column(int64_t m, double* Q, const int64_t* use, int64_t nuse, int64_t c) {
    int64_t best = 0;
    double bres = -1.0;
    for (int64_t i = 0; i < m; ++i) {
        double acc = 0.0;
        for (int64_t t = 0; t < nuse; ++t) acc += Q[i + m * use[t]] * Q[i + m * use[t]];
        const double res = 1.0 - acc;
        if (res > bres) { bres = res; best = i; }
    }
    double* u = Q + m * c;
    for (int64_t r = 0; r < m; ++r) u[r] = (r == best) ? 1.0 : 0.0;
    for (int pass = 0; pass < 2; ++pass)
        for (int64_t t = 0; t < nuse; ++t) {
            const double* w = Q + m * use[t];
            double d = 0.0;
            for (int64_t r = 0; r < m; ++r) d += w[r] * u[r];
            for (int64_t r = 0; r < m; ++r) u[r] -= d * w[r];
        }
    double nn = 0.0;
    for (int64_t r = 0; r < m; ++r) nn += u[r] * u[r];
    nn = sqrt(nn);
    for (int64_t r = 0; r < m; ++r) u[r] /= nn;
}

int or_jacobi_svd(int64_t m, int64_t n, const double* A, int64_t lda, double* U, double* s, double* V, int max_sweeps) {
    int trans = m < n;
    int64_t mm = trans ? n : m; /* rows of the tall working matrix */
    int64_t p = trans ? m : n;  /* its columns = min(m,n) */
    double* W = (double*)malloc(sizeof(double) * mm * p);
    double* Q = (double*)malloc(sizeof(double) * p * p);
    for (int64_t c = 0; c < p; ++c)
        for (int64_t r = 0; r < mm; ++r) W[r + mm * c] = trans ? A[c + lda * r] : A[r + lda * c];
    double tol = (double)mm * ldexp(1.0, -53);
    int sweeps = jacobi_tall(mm, p, W, Q, max_sweeps, tol);

    /* singular values = column norms; order descending (stable in index) */
    double* sv = (double*)malloc(sizeof(double) * p);
    int64_t* ord = (int64_t*)malloc(sizeof(int64_t) * p);
    for (int64_t c = 0; c < p; ++c) {
        double acc = 0.0;
        for (int64_t r = 0; r < mm; ++r) acc += W[r + mm * c] * W[r + mm * c];
        sv[c] = sqrt(acc);
        ord[c] = c;
    }
    for (int64_t a = 1; a < p; ++a) { /* insertion sort */
        int64_t key = ord[a], b = a - 1;
        while (b >= 0 && sv[ord[b]] < sv[key]) { ord[b + 1] = ord[b]; --b; }
        ord[b + 1] = key;
    }
    /* left vectors of the tall problem (mm x p) and its right vectors (p x p) */
    double* Lt = (double*)malloc(sizeof(double) * mm * p);
    double* Rt = (double*)malloc(sizeof(double) * p * p);
    for (int64_t c = 0; c < p; ++c) {
        int64_t o = ord[c];
        for (int64_t r = 0; r < mm; ++r) Lt[r + mm * c] = (sv[o] > 0.0) ? W[r + mm * o] / sv[o] : 0.0;
        for (int64_t r = 0; r < p; ++r) Rt[r + p * c] = Q[r + p * o];
    }
    /* zero singular values: complete the left vector (complement_column) against
     * the columns with nonzero singular values and the zero ones before it */
    {
        int64_t* use = (int64_t*)malloc(sizeof(int64_t) * (p > 0 ? p : 1));
        for (int64_t c = 0; c < p; ++c) {
            if (sv[ord[c]] > 0.0) continue;
            int64_t nuse = 0;
            for (int64_t q = 0; q < p; ++q)
                if (q != c && !(sv[ord[q]] == 0.0 && q > c)) use[nuse++] = q;
            complement_column(mm, Lt, use, nuse, c);
        }
        free(use);
    }
    /* Undo the transpose: A = Lt S Rt^T (tall) or A^T = Lt S Rt^T (wide). */
    double* Uo = trans ? Rt : Lt; int64_t ldu = trans ? p : mm;
    double* Vo = trans ? Lt : Rt; int64_t ldv = trans ? mm : p;
    /* sign convention on the left vectors */
    for (int64_t c = 0; c < p; ++c) {
        int64_t best = 0;
        for (int64_t r = 1; r < m; ++r)
            if (fabs(Uo[r + ldu * c]) > fabs(Uo[best + ldu * c])) best = r;
        if (Uo[best + ldu * c] < 0.0) {
            for (int64_t r = 0; r < m; ++r) Uo[r + ldu * c] = -Uo[r + ldu * c];
            for (int64_t r = 0; r < n; ++r) Vo[r + ldv * c] = -Vo[r + ldv * c];
        }
    }
    if (U) for (int64_t c = 0; c < p; ++c) for (int64_t r = 0; r < m; ++r) U[r + m * c] = Uo[r + ldu * c];
    if (V) for (int64_t c = 0; c < p; ++c) for (int64_t r = 0; r < n; ++r) V[r + n * c] = Vo[r + ldv * c];
    if (s) for (int64_t c = 0; c < p; ++c) s[c] = sv[ord[c]];
    free(W); free(Q); free(sv); free(ord); free(Lt); free(Rt);
    return sweeps;
}

/* ------------------------------------------------------------------------- */
/* Theorem 4 (DCT-based t-SVD), computed as the paper prescribes: DCT along  */
/* the tubes, then the SVD of every frontal slice of Xbar.  Thin factors,    */
/* p = min(n1,n2), in the transform domain:                                  */
/*   Ubar n1 x p x n3, Sbar p x n3 (column k = singular values of slice k),  */
/*   Vbar n2 x p x n3.  Returns the largest sweep count, or -1.              */
/* ------------------------------------------------------------------------- */
/* The slice SVDs are independent: slices are split over the host threads. */
struct svd_ctx { int64_t n1, n2, p; const double* Xb; double *U, *S, *V; int max_sweeps; int* sweeps; };
static void svd_range(void* a, int64_t k0, int64_t k1) {
    const struct svd_ctx* c = (const struct svd_ctx*)a;
    for (int64_t k = k0; k < k1; ++k)
        c->sweeps[k] = or_jacobi_svd(c->n1, c->n2, c->Xb + k * c->n1 * c->n2, c->n1, c->U ? c->U + k * c->n1 * c->p : NULL,
                                     c->S + k * c->p, c->V ? c->V + k * c->n2 * c->p : NULL, c->max_sweeps);
}
static int worst_sweeps(const int* sw, int64_t n) {
    int worst = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (sw[k] < 0) worst = -1;
        else if (worst >= 0 && sw[k] > worst) worst = sw[k];
    }
    return worst;
}

int or_tsvd_dct(int64_t n1, int64_t n2, int64_t n3, const double* X, double* Ubar, double* Sbar, double* Vbar,
                int max_sweeps) {
    int64_t p = n1 < n2 ? n1 : n2;
    double* Xb = (double*)malloc(sizeof(double) * n1 * n2 * n3);
    int* sw = (int*)malloc(sizeof(int) * n3);
    or_dct_tubes(n1, n2, n3, X, Xb);
    struct svd_ctx c = {n1, n2, p, Xb, Ubar, Sbar, Vbar, max_sweeps, sw};
    parallel_for(n3, svd_range, &c);
    int worst = worst_sweeps(sw, n3);
    free(Xb);
    free(sw);
    return worst;
}

/* ------------------------------------------------------------------------- */
/* Theorem 4 with full factors: U m1 x m1, V m2 x m2 orthogonal per slice.    */
/* The thin factors as in or_tsvd_dct; the side with more rows than p         */
/* (U if n1 > n2, V if n2 > n1) is completed to an orthonormal basis column   */
/* by column (complement_column against every column so far), each new       */
/* column with its largest-magnitude entry (first one on ties) positive.      */
/* Returns the largest sweep count, or -1.                                    */
/* ------------------------------------------------------------------------- */
static void complete_columns(int64_t m, int64_t p, double* Q) {
    int64_t* use = (int64_t*)malloc(sizeof(int64_t) * m);
    for (int64_t c = p; c < m; ++c) {
        for (int64_t q = 0; q < c; ++q) use[q] = q;
        complement_column(m, Q, use, c, c);
        double* u = Q + m * c;
        int64_t best = 0;
        for (int64_t r = 1; r < m; ++r) if (fabs(u[r]) > fabs(u[best])) best = r;
        if (u[best] < 0.0) for (int64_t r = 0; r < m; ++r) u[r] = -u[r];
    }
    free(use);
}

struct svdf_ctx { int64_t n1, n2, p; const double* Xb; double *U, *S, *V; int max_sweeps; int* sweeps; };
static void svdf_range(void* a, int64_t k0, int64_t k1) {
    const struct svdf_ctx* c = (const struct svdf_ctx*)a;
    const int64_t n1 = c->n1, n2 = c->n2, p = c->p;
    for (int64_t k = k0; k < k1; ++k) {
        double* U = c->U + k * n1 * n1;
        double* V = c->V + k * n2 * n2;
        /* thin factors into the first p columns (leading dimensions n1 and n2) */
        c->sweeps[k] = or_jacobi_svd(n1, n2, c->Xb + k * n1 * n2, n1, U, c->S + k * p, V, c->max_sweeps);
        if (n1 > p) complete_columns(n1, p, U);
        if (n2 > p) complete_columns(n2, p, V);
    }
}

int or_tsvd_dct_full(int64_t n1, int64_t n2, int64_t n3, const double* X, double* Ubar, double* Sbar, double* Vbar,
                     int max_sweeps) {
    int64_t p = n1 < n2 ? n1 : n2;
    double* Xb = (double*)malloc(sizeof(double) * n1 * n2 * n3);
    int* sw = (int*)malloc(sizeof(int) * n3);
    or_dct_tubes(n1, n2, n3, X, Xb);
    struct svdf_ctx c = {n1, n2, p, Xb, Ubar, Sbar, Vbar, max_sweeps, sw};
    parallel_for(n3, svdf_range, &c);
    int worst = worst_sweeps(sw, n3);
    free(Xb);
    free(sw);
    return worst;
}

/* ------------------------------------------------------------------------- */
/* Theorem 5 (tensor singular value thresholding) with Algorithm 1's loop    */
/* body: Zbar = dct(Z); per slice SVD; Dbar = (Sbar - tau)_+; rebuild         */
/* Ubar Dbar Vbar^T; Y = idct.  ranks[k] = #{sigma > tau} (may be NULL).      */
/* Returns the largest sweep count, or -1.                                    */
/* ------------------------------------------------------------------------- */
/* One transform-domain slice of the t-SVT: SVD, (sigma - tau)_+, rebuild. */
static int svt_slice(int64_t n1, int64_t n2, const double* Zk, double tau, double* Yk, int32_t* rank, int max_sweeps) {
    int64_t p = n1 < n2 ? n1 : n2;
    double* U = (double*)malloc(sizeof(double) * n1 * p);
    double* V = (double*)malloc(sizeof(double) * n2 * p);
    double* sv = (double*)malloc(sizeof(double) * p);
    int sw = or_jacobi_svd(n1, n2, Zk, n1, U, sv, V, max_sweeps);
    int32_t r = 0;
    for (int64_t c = 0; c < p; ++c) if (sv[c] > tau) ++r;
    if (rank) *rank = r;
    for (int64_t j = 0; j < n2; ++j)
        for (int64_t i = 0; i < n1; ++i) {
            double acc = 0.0;
            for (int64_t c = 0; c < p; ++c) {
                double d = sv[c] - tau;
                if (d > 0.0) acc += U[i + n1 * c] * d * V[j + n2 * c];
            }
            Yk[i + n1 * j] = acc;
        }
    free(U); free(V); free(sv);
    return sw;
}
struct svt_ctx { int64_t n1, n2; const double* Zb; double* Yb; double tau; int32_t* ranks; int max_sweeps; int* sweeps; };
static void svt_range(void* a, int64_t k0, int64_t k1) {
    const struct svt_ctx* c = (const struct svt_ctx*)a;
    const int64_t s = c->n1 * c->n2;
    for (int64_t k = k0; k < k1; ++k)
        c->sweeps[k] = svt_slice(c->n1, c->n2, c->Zb + k * s, c->tau, c->Yb + k * s, c->ranks ? c->ranks + k : NULL,
                                 c->max_sweeps);
}

int or_tsvt_dct(int64_t n1, int64_t n2, int64_t n3, const double* Z, double tau, double* Y, int32_t* ranks,
                int max_sweeps) {
    int64_t s = n1 * n2;
    double* Zb = (double*)malloc(sizeof(double) * s * n3);
    double* Yb = (double*)malloc(sizeof(double) * s * n3);
    int* sw = (int*)malloc(sizeof(int) * n3);
    or_dct_tubes(n1, n2, n3, Z, Zb);
    struct svt_ctx c = {n1, n2, Zb, Yb, tau, ranks, max_sweeps, sw};
    parallel_for(n3, svt_range, &c);
    int worst = worst_sweeps(sw, n3);
    or_idct_tubes(n1, n2, n3, Yb, Y);
    free(Zb); free(Yb); free(sw);
    return worst;
}

/* Section 4, TNN-C: (1/n3) sum_k ||Xbar^(k)||_*  (nuclear norm of each slice). */
double or_tnn_c(int64_t n1, int64_t n2, int64_t n3, const double* X, int max_sweeps) {
    int64_t p = n1 < n2 ? n1 : n2;
    double* Sb = (double*)malloc(sizeof(double) * p * n3);
    or_tsvd_dct(n1, n2, n3, X, NULL, Sb, NULL, max_sweeps);
    double acc = 0.0;
    for (int64_t e = 0; e < p * n3; ++e) acc += Sb[e];
    free(Sb);
    return acc / (double)n3;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 1 (ADMM for TNN-C completion), with the penalty given per       */
/* iteration: iteration l uses beta[l] in Z = X - M/beta, in the X-update    */
/* and in the multiplier update, and thresholds at tau[l] (Algorithm 1 uses  */
/* tau = 1/beta).  mask[e] != 0 marks the observed set Omega.                */
/* X, M: in = initial iterates (X normally B on Omega), out = final.          */
/* Stops after iteration l when ||X_new - X_old||_F / ||X_old||_F <= tol      */
/* (tol <= 0: run all L iterations).  Returns the number of iterations run;   */
/* *relchg gets the last relative change.                                     */
/* ------------------------------------------------------------------------- */
int or_complete(int64_t n1, int64_t n2, int64_t n3, const double* B, const uint8_t* mask, int L,
                const double* beta, const double* tau, double tol, int max_sweeps, double* X, double* M,
                double* relchg) {
    int64_t N = n1 * n2 * n3;
    double* Z = (double*)malloc(sizeof(double) * N);
    double* Y = (double*)malloc(sizeof(double) * N);
    int it = 0;
    double rc = 0.0;
    for (int l = 0; l < L; ++l) {
        double b = beta[l];
        for (int64_t e = 0; e < N; ++e) Z[e] = X[e] - M[e] / b;                 /* line: Z = X - M/beta */
        or_tsvt_dct(n1, n2, n3, Z, tau[l], Y, NULL, max_sweeps);                /* Y-subproblem, Theorem 5 */
        double dn = 0.0, xn = 0.0;
        for (int64_t e = 0; e < N; ++e) {
            double xnew = mask[e] ? B[e] : Y[e] + M[e] / b;                     /* X-update closed form */
            M[e] = M[e] + b * (Y[e] - xnew);                                    /* multiplier update */
            dn += (xnew - X[e]) * (xnew - X[e]);
            xn += X[e] * X[e];
            X[e] = xnew;
        }
        ++it;
        rc = (xn > 0.0) ? sqrt(dn / xn) : sqrt(dn);
        if (tol > 0.0 && rc <= tol) break;
    }
    if (relchg) *relchg = rc;
    free(Z); free(Y);
    return it;
}

/* ------------------------------------------------------------------------- */
/* Section 6 (concluding remarks): other invertible transforms along the     */
/* tubes in place of the DCT.  With a transform matrix L (row-major n3 x n3) */
/* and its inverse Linv (supplied by the caller):                             */
/*   Zbar(:,:,k) = sum_t L[k][t] Z(:,:,t),  Ybar^(k) = U (S - tau)_+ V^T of   */
/*   Zbar^(k),  Y(:,:,t) = sum_k Linv[t][k] Ybar(:,:,k).                      */
/* With L = C (orthonormal DCT-II) this is or_tsvt_dct.                       */
/* ------------------------------------------------------------------------- */
int or_tsvt_transform(int64_t n1, int64_t n2, int64_t n3, const double* L, const double* Linv, const double* Z,
                      double tau, double* Y, int32_t* ranks, int max_sweeps) {
    int64_t s = n1 * n2;
    double* Zb = (double*)malloc(sizeof(double) * s * n3);
    double* Yb = (double*)malloc(sizeof(double) * s * n3);
    int* sw = (int*)malloc(sizeof(int) * n3);
    tube_apply(n1, n2, n3, L, 0, Z, Zb);
    struct svt_ctx c = {n1, n2, Zb, Yb, tau, ranks, max_sweeps, sw};
    parallel_for(n3, svt_range, &c);
    int worst = worst_sweeps(sw, n3);
    tube_apply(n1, n2, n3, Linv, 0, Yb, Y);
    free(Zb); free(Yb); free(sw);
    return worst;
}

/* ------------------------------------------------------------------------- */
/* Section 2: the DFT-based t-SVD and TNN-F (complex arithmetic, C99).        */
/* Xt = fft(X,[],3), the unnormalized DFT along every tube:                   */
/*   Xt(i,j,k) = sum_t X(i,j,t) exp(-2 pi i k t / n3),                        */
/* written out from the definition (O(n3^2) per tube).  The angle k t is     */
/* reduced modulo n3 in integers before the cosine and sine.                  */
/* ------------------------------------------------------------------------- */

static void dft_twiddle(int64_t n, int64_t k, int64_t t, double sgn, double* re, double* im) {
    const double pi = acos(-1.0);
    const int64_t q = (k * t) % n;
    const double a = 2.0 * pi * (double)q / (double)n;
    *re = cos(a);
    *im = sgn * sin(a);
}

/* Real input X; output real and imaginary parts (same layout). */
void or_dft_tubes(int64_t n1, int64_t n2, int64_t n3, const double* X, double* Xr, double* Xi) {
    for (int64_t j = 0; j < n2; ++j)
        for (int64_t i = 0; i < n1; ++i)
            for (int64_t k = 0; k < n3; ++k) {
                double ar = 0.0, ai = 0.0;
                for (int64_t t = 0; t < n3; ++t) {
                    double wr, wi;
                    dft_twiddle(n3, k, t, -1.0, &wr, &wi);
                    const double x = X[X3(i, j, t, n1, n2)];
                    ar += wr * x;
                    ai += wi * x;
                }
                Xr[X3(i, j, k, n1, n2)] = ar;
                Xi[X3(i, j, k, n1, n2)] = ai;
            }
}

/* Inverse DFT along tubes, X(i,j,t) = (1/n3) sum_k Xt(i,j,k) exp(2 pi i k t / n3),
 * of complex input (Xr, Xi); outputs real and imaginary parts. */
void or_idft_tubes(int64_t n1, int64_t n2, int64_t n3, const double* Xr, const double* Xi, double* Yr, double* Yi) {
    for (int64_t j = 0; j < n2; ++j)
        for (int64_t i = 0; i < n1; ++i)
            for (int64_t t = 0; t < n3; ++t) {
                double ar = 0.0, ai = 0.0;
                for (int64_t k = 0; k < n3; ++k) {
                    double wr, wi;
                    dft_twiddle(n3, k, t, 1.0, &wr, &wi);
                    const double xr = Xr[X3(i, j, k, n1, n2)], xi = Xi[X3(i, j, k, n1, n2)];
                    ar += wr * xr - wi * xi;
                    ai += wr * xi + wi * xr;
                }
                Yr[X3(i, j, t, n1, n2)] = ar / (double)n3;
                Yi[X3(i, j, t, n1, n2)] = ai / (double)n3;
            }
}

/* Equation (bcirc): the block circulant matrix of X, (n1 n3) x (n2 n3),      */
/* column-major; block (r, c) is X^(((r - c) mod n3) + 1).                     */
void or_bcirc(int64_t n1, int64_t n2, int64_t n3, const double* X, double* M) {
    const int64_t ld = n1 * n3;
    for (int64_t bc = 0; bc < n3; ++bc)
        for (int64_t br = 0; br < n3; ++br) {
            const int64_t k = ((br - bc) % n3 + n3) % n3;
            for (int64_t j = 0; j < n2; ++j)
                for (int64_t i = 0; i < n1; ++i) M[(br * n1 + i) + ld * (bc * n2 + j)] = X[X3(i, j, k, n1, n2)];
        }
}

/* One-sided Jacobi SVD of a complex m x n matrix (Hestenes; complex columns).
 * For the pair (x, y) with alpha = |x|^2, beta = |y|^2, gamma = x^H y =
 * |gamma| e^{i phi}: y is first multiplied by e^{-i phi}, which makes the
 * pair's inner product real (|gamma|), then the real rotation of the real case
 * is applied: zeta = (beta - alpha) / (2 |gamma|), t = sgn(zeta) / (|zeta| +
 * sqrt(1 + zeta^2)), c = 1/sqrt(1 + t^2), s = c t.  The same unitary acts on
 * the columns of V.  Rotation test |gamma| > tol sqrt(alpha beta), tol = m u.
 * Works on A (tall form: A itself if m >= n, else A^H); returns the sweeps
 * (-1 at the limit).  Outputs for the tall form: W (mm x p, columns sigma_j
 * u_j, unsorted) and Q (p x p) with A_tall Q = W. */
static int jacobi_tall_c(int64_t m, int64_t n, double* Wr, double* Wi, double* Vr, double* Vi, int max_sweeps,
                         double tol) {
    /* complex values as separate real and imaginary arrays, same layout */
    for (int64_t c = 0; c < n; ++c)
        for (int64_t r = 0; r < n; ++r) {
            Vr[r + n * c] = (r == c) ? 1.0 : 0.0;
            Vi[r + n * c] = 0.0;
        }
    for (int sweep = 1; sweep <= max_sweeps; ++sweep) {
        int64_t rotations = 0;
        for (int64_t i = 0; i < n - 1; ++i)
            for (int64_t j = i + 1; j < n; ++j) {
                double *xr = Wr + m * i, *xi = Wi + m * i, *yr = Wr + m * j, *yi = Wi + m * j;
                double alpha = 0.0, beta = 0.0, gr = 0.0, gi = 0.0;
                for (int64_t r = 0; r < m; ++r) {
                    alpha += xr[r] * xr[r] + xi[r] * xi[r];
                    beta += yr[r] * yr[r] + yi[r] * yi[r];
                    /* gamma = conj(x) . y */
                    gr += xr[r] * yr[r] + xi[r] * yi[r];
                    gi += xr[r] * yi[r] - xi[r] * yr[r];
                }
                const double ag = sqrt(gr * gr + gi * gi);
                if (ag == 0.0 || ag <= tol * sqrt(alpha * beta)) continue;
                const double pr = gr / ag, pi = -gi / ag; /* e^{-i phi} = conj(gamma) / |gamma| */
                double zeta = (beta - alpha) / (2.0 * ag);
                double sgn = (zeta >= 0.0) ? 1.0 : -1.0;
                double t = sgn / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                double c = 1.0 / sqrt(1.0 + t * t);
                double s = c * t;
                for (int64_t r = 0; r < m; ++r) {
                    const double ar = xr[r], ai = xi[r];
                    const double br = yr[r] * pr - yi[r] * pi, bi = yr[r] * pi + yi[r] * pr; /* y e^{-i phi} */
                    xr[r] = c * ar - s * br; xi[r] = c * ai - s * bi;
                    yr[r] = s * ar + c * br; yi[r] = s * ai + c * bi;
                }
                double *ur = Vr + n * i, *ui = Vi + n * i, *wr = Vr + n * j, *wi = Vi + n * j;
                for (int64_t r = 0; r < n; ++r) {
                    const double ar = ur[r], ai = ui[r];
                    const double br = wr[r] * pr - wi[r] * pi, bi = wr[r] * pi + wi[r] * pr;
                    ur[r] = c * ar - s * br; ui[r] = c * ai - s * bi;
                    wr[r] = s * ar + c * br; wi[r] = s * ai + c * bi;
                }
                ++rotations;
            }
        if (rotations == 0) return sweep;
    }
    return -1;
}

/* Singular values (descending) of a complex m x n matrix (column-major,
 * real and imaginary parts); optionally its thresholded rebuild
 * Y = U (S - tau)_+ V^H (Yr, Yi may be NULL).  Returns the sweeps. */
int or_jacobi_svt_c(int64_t m, int64_t n, const double* Ar, const double* Ai, double tau, double* s, double* Yr,
                    double* Yi, int32_t* rank, int max_sweeps) {
    const int trans = m < n;
    const int64_t mm = trans ? n : m, p = trans ? m : n;
    double* Wr = (double*)malloc(sizeof(double) * mm * p);
    double* Wi = (double*)malloc(sizeof(double) * mm * p);
    double* Qr = (double*)malloc(sizeof(double) * p * p);
    double* Qi = (double*)malloc(sizeof(double) * p * p);
    for (int64_t c = 0; c < p; ++c)
        for (int64_t r = 0; r < mm; ++r) {
            /* tall form: A (m >= n) or A^H */
            const int64_t e = trans ? c + m * r : r + m * c;
            Wr[r + mm * c] = Ar[e];
            Wi[r + mm * c] = trans ? -Ai[e] : Ai[e];
        }
    const int sweeps = jacobi_tall_c(mm, p, Wr, Wi, Qr, Qi, max_sweeps, (double)mm * ldexp(1.0, -53));
    double* sv = (double*)malloc(sizeof(double) * p);
    for (int64_t c = 0; c < p; ++c) {
        double acc = 0.0;
        for (int64_t r = 0; r < mm; ++r) acc += Wr[r + mm * c] * Wr[r + mm * c] + Wi[r + mm * c] * Wi[r + mm * c];
        sv[c] = sqrt(acc);
    }
    int32_t rk = 0;
    for (int64_t c = 0; c < p; ++c) if (sv[c] > tau) ++rk;
    if (rank) *rank = rk;
    if (s) { /* descending, by repeated selection */
        char* used = (char*)calloc((size_t)p, 1);
        for (int64_t o = 0; o < p; ++o) {
            int64_t best = -1;
            for (int64_t c = 0; c < p; ++c)
                if (!used[c] && (best < 0 || sv[c] > sv[best])) best = c;
            used[best] = 1;
            s[o] = sv[best];
        }
        free(used);
    }
    if (Yr) {
        /* tall form A_t = W Q^H with columns W(:,c) = sigma_c u_c; thresholded:
         * sum_c W(:,c) ((sigma_c - tau)/sigma_c) conj(Q(:,c))^T.  Element (i, j)
         * of A is element (i, j) of A_t (m >= n) or conj of element (j, i). */
        for (int64_t j = 0; j < n; ++j)
            for (int64_t i = 0; i < m; ++i) {
                double accr = 0.0, acci = 0.0;
                for (int64_t c = 0; c < p; ++c) {
                    const double d = sv[c] - tau;
                    if (d <= 0.0) continue;
                    const double f = d / sv[c];
                    const int64_t a = trans ? j : i, b = trans ? i : j; /* (row of W, row of Q) */
                    const double wr = Wr[a + mm * c], wi = Wi[a + mm * c];
                    const double qr = Qr[b + p * c], qi = -Qi[b + p * c]; /* conj(Q) */
                    accr += f * (wr * qr - wi * qi);
                    acci += f * (wr * qi + wi * qr);
                }
                Yr[i + m * j] = accr;
                Yi[i + m * j] = trans ? -acci : acci;
            }
    }
    free(Wr); free(Wi); free(Qr); free(Qi); free(sv);
    return sweeps;
}

/* Slice-wise complex t-SVT in the Fourier domain (Lu et al.'s TNN-F t-SVT,
 * the DFT counterpart of Theorem 5): Zt = fft(Z,[],3); every slice k gets
 * Yt^(k) = U (S - tau)_+ V^H; Y = ifft(Yt).  Y is real for real Z (conjugate
 * slices give conjugate results); the largest |imaginary part| of the
 * inverse transform is returned in *max_imag.  ranks[k] (may be NULL).
 * Returns the largest sweep count, or -1. */
struct svtc_ctx { int64_t n1, n2; const double *Zr, *Zi; double *Yr, *Yi; double tau; int32_t* ranks; int max_sweeps; int* sw; };
static void svtc_range(void* a, int64_t k0, int64_t k1) {
    const struct svtc_ctx* c = (const struct svtc_ctx*)a;
    const int64_t s = c->n1 * c->n2;
    for (int64_t k = k0; k < k1; ++k)
        c->sw[k] = or_jacobi_svt_c(c->n1, c->n2, c->Zr + k * s, c->Zi + k * s, c->tau, NULL, c->Yr + k * s,
                                   c->Yi + k * s, c->ranks ? c->ranks + k : NULL, c->max_sweeps);
}

int or_tsvt_dft(int64_t n1, int64_t n2, int64_t n3, const double* Z, double tau, double* Y, int32_t* ranks,
                double* max_imag, int max_sweeps) {
    const int64_t N = n1 * n2 * n3;
    double* Zr = (double*)malloc(sizeof(double) * N);
    double* Zi = (double*)malloc(sizeof(double) * N);
    double* Yr = (double*)malloc(sizeof(double) * N);
    double* Yi = (double*)malloc(sizeof(double) * N);
    double* Ti = (double*)malloc(sizeof(double) * N);
    int* sw = (int*)malloc(sizeof(int) * n3);
    or_dft_tubes(n1, n2, n3, Z, Zr, Zi);
    struct svtc_ctx c = {n1, n2, Zr, Zi, Yr, Yi, tau, ranks, max_sweeps, sw};
    parallel_for(n3, svtc_range, &c);
    or_idft_tubes(n1, n2, n3, Yr, Yi, Y, Ti);
    double mi = 0.0;
    for (int64_t e = 0; e < N; ++e) if (fabs(Ti[e]) > mi) mi = fabs(Ti[e]);
    if (max_imag) *max_imag = mi;
    int worst = worst_sweeps(sw, n3);
    free(Zr); free(Zi); free(Yr); free(Yi); free(Ti); free(sw);
    return worst;
}

/* Section 2, TNN-F: (1/n3) sum_k ||Xt^(k)||_* over the unnormalized DFT slices. */
double or_tnn_f(int64_t n1, int64_t n2, int64_t n3, const double* X, int max_sweeps) {
    const int64_t N = n1 * n2 * n3, s = n1 * n2, p = n1 < n2 ? n1 : n2;
    double* Xr = (double*)malloc(sizeof(double) * N);
    double* Xi = (double*)malloc(sizeof(double) * N);
    double* sv = (double*)malloc(sizeof(double) * p);
    or_dft_tubes(n1, n2, n3, X, Xr, Xi);
    double acc = 0.0;
    for (int64_t k = 0; k < n3; ++k) {
        or_jacobi_svt_c(n1, n2, Xr + k * s, Xi + k * s, 0.0, sv, NULL, NULL, NULL, max_sweeps);
        for (int64_t c = 0; c < p; ++c) acc += sv[c];
    }
    free(Xr); free(Xi); free(sv);
    return acc / (double)n3;
}
