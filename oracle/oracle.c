/*
 * CPU oracle for inverse iteration with compact-WY re-orthogonalization.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, obviously correct
 * FP64 reference of what the GPU library computes.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * library never links, loads or calls it.  It shares no code, header, table or
 * helper with the HIP path.
 *
 * Method: H. Ishigami, K. Kimura, Y. Nakamura, "On Implementation and
 * Evaluation of Inverse Iteration Algorithm with compact WY Orthogonalization"
 * (arXiv:1209.1910).  Every function names the passage it follows.  Where the
 * paper is silent (how eigenvalues are bisected, which tridiagonal solver,
 * random start vectors, the stop rule) the function says which reading it
 * takes; the readings are the same ones the GPU library documents.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math, no FMA), so
 * every floating-point operation is one IEEE binary64 round-to-nearest step
 * in the order written.
 *
 * Parity status: every exported function is pinned by the CPU tests against
 * closed forms, brute force, library routines on special cases, or exact
 * identities of the paper; none is "parity unpinned".
 */
#include <float.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------- */
/* Setup: norm, cluster tolerance, Sturm pivot floor, bisection bracket.       */
/* ------------------------------------------------------------------------- */

typedef struct {
    double norm1;   /* ||T||_1 = max_i (|d_i| + |e_{i-1}|) + |e_i|               */
    double tol;     /* 1e-3 * ||T||_1: Peters-Wilkinson gap (section 2.1)        */
    double pivmin;  /* Sturm-count floor: DBL_MIN * max(1, max_i e_i^2)          */
    double pivthr;  /* LU pivot floor: DBL_EPSILON * ||T||_1                      */
    double gl, gu;  /* widened Gershgorin bracket: count(gl) = 0, count(gu) = n  */
    double tnorm;   /* max(|gl|, |gu|) of the unwidened Gershgorin interval       */
} or_params;

int or_sturm_count(int n, const double *d, const double *e2, double pivmin, double sigma);

/* The paper clusters eigenvalues whose distance is at most 1e-3 ||T||
 * (section 2.1, and the test in Alg. 4); ||T|| is read as the 1-norm, which
 * for a symmetric matrix equals the infinity norm. */
int or_setup(int n, const double *d, const double *e, or_params *p)
{
    if (n < 1 || !d || !p) return -1;
    double norm1 = 0.0, maxe2 = 0.0, gl = 0.0, gu = 0.0;
    for (int i = 0; i < n; i++) {
        double r = fabs(d[i]);
        double s = 0.0;
        if (i > 0) { r = r + fabs(e[i - 1]); s = s + fabs(e[i - 1]); }
        if (i < n - 1) { r = r + fabs(e[i]); s = s + fabs(e[i]); }
        double lo = d[i] - s, hi = d[i] + s;
        if (i == 0 || r > norm1) norm1 = r;
        if (i == 0 || lo < gl) gl = lo;
        if (i == 0 || hi > gu) gu = hi;
    }
    for (int i = 0; i < n - 1; i++) {
        double q = e[i] * e[i];
        if (q > maxe2) maxe2 = q;
    }
    p->norm1 = norm1;
    p->tol = 1.0e-3 * norm1;
    p->pivmin = DBL_MIN * (maxe2 > 1.0 ? maxe2 : 1.0);
    p->pivthr = DBL_EPSILON * norm1;
    double tnorm = fabs(gl) > fabs(gu) ? fabs(gl) : fabs(gu);
    p->tnorm = tnorm;

    double *e2 = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    if (!e2) return -2;
    for (int i = 0; i < n - 1; i++) e2[i] = e[i] * e[i];
    double w = (2.0 * DBL_EPSILON * tnorm) * (double)n + 2.0 * p->pivmin;
    double lo = gl - w, hi = gu + w;
    for (int t = 0; t < 64; t++) {
        lo = gl - w;
        hi = gu + w;
        if (or_sturm_count(n, d, e2, p->pivmin, lo) == 0 &&
            or_sturm_count(n, d, e2, p->pivmin, hi) == n)
            break;
        w = 2.0 * w;
    }
    free(e2);
    p->gl = lo;
    p->gu = hi;
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Eigenvalues by bisection (the experiments take them from LAPACK's         */
/* bisection routine, section 5.1; the recurrence below is the classical     */
/* Sturm count of T - sigma I).                                              */
/* ------------------------------------------------------------------------- */

/* Number of eigenvalues of T strictly below sigma: the number of negative
 * pivots of the LDL^T factorization of T - sigma I, with pivots of magnitude
 * at most pivmin replaced by -pivmin. */
int or_sturm_count(int n, const double *d, const double *e2, double pivmin, double sigma)
{
    double q = d[0] - sigma;
    if (fabs(q) <= pivmin) q = -pivmin;
    int cnt = q < 0.0 ? 1 : 0;
    for (int i = 1; i < n; i++) {
        double t1 = d[i] - sigma;
        double t2 = e2[i - 1] / q;
        q = t1 - t2;
        if (fabs(q) <= pivmin) q = -pivmin;
        if (q < 0.0) cnt++;
    }
    return cnt;
}

/* lambda_k for k = il..iu (1-based, inclusive) into W[0..iu-il].
 * Plain bisection from [gl, gu] until the bracket is at most
 * 2 eps tnorm wide (at most 128 halvings); the value is the bracket midpoint. */
int or_bisect(int n, const double *d, const double *e, int il, int iu, double *W)
{
    if (n < 1 || il < 1 || iu < il || iu > n) return -1;
    or_params p;
    if (or_setup(n, d, e, &p)) return -2;
    double *e2 = (double *)malloc(sizeof(double) * (size_t)(n > 1 ? n - 1 : 1));
    if (!e2) return -2;
    for (int i = 0; i < n - 1; i++) e2[i] = e[i] * e[i];
    double atol = 2.0 * DBL_EPSILON * p.tnorm;
    for (int k = il; k <= iu; k++) {
        double lo = p.gl, hi = p.gu;
        for (int it = 0; it < 128 && (hi - lo) > atol; it++) {
            double mid = lo + 0.5 * (hi - lo);
            if (or_sturm_count(n, d, e2, p.pivmin, mid) >= k) hi = mid;
            else lo = mid;
        }
        W[k - il] = lo + 0.5 * (hi - lo);
    }
    free(e2);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Peters-Wilkinson clusters (section 2.1, Alg. 1 and Alg. 4): eigenvalue j */
/* joins the cluster of j-1 when lambda_j - lambda_{j-1} <= tol.             */
/* ------------------------------------------------------------------------- */

int or_clusters(int m, const double *W, double tol, int *start, int *size)
{
    int ncl = 0;
    for (int j = 0; j < m; j++) {
        if (j == 0 || (W[j] - W[j - 1]) > tol) {
            start[ncl] = j;
            size[ncl] = 1;
            ncl++;
        } else {
            size[ncl - 1]++;
        }
    }
    return ncl;
}

/* ------------------------------------------------------------------------- */
/* Random start vectors (Alg. 1 and Alg. 4 start each v^(0) at random).      */
/* Reading: entry i of the start vector of global eigenvalue index k is       */
/* 2u - 1 with u = (z >> 11) 2^-53 and z the (key+1)-th output of a           */
/* SplitMix64 stream (Steele, Lea, Flood, OOPSLA 2014) seeded with `seed`,    */
/* key = (k << 32) | i.                                                       */
/* ------------------------------------------------------------------------- */

uint64_t or_splitmix64(uint64_t seed, uint64_t index)
{
    /* index-th output (1-based) of the SplitMix64 stream seeded with `seed` */
    uint64_t z = seed + index * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

void or_start_vector(uint64_t seed, int64_t kglob, int n, double *v)
{
    for (int i = 0; i < n; i++) {
        uint64_t key = ((uint64_t)kglob << 32) | (uint64_t)(uint32_t)i;
        uint64_t z = or_splitmix64(seed, key + 1);
        double u = (double)(z >> 11) * (1.0 / 9007199254740992.0);
        v[i] = 2.0 * u - 1.0;
    }
}

/* ------------------------------------------------------------------------- */
/* Solving (T - lambda I) v^(k) = v^(k-1) (Eq. (1)).  Reading: Gaussian        */
/* elimination with partial pivoting on the tridiagonal matrix, giving        */
/* P (T - sigma I) = L U with U upper triangular with three diagonals          */
/* (u1, u2, u3) and unit lower bidiagonal L (multipliers l).  A pivot of      */
/* magnitude below pivthr is replaced by +-pivthr (sign of the pivot, + for 0); */
/* returns how many pivots were replaced.                                      */
/* ------------------------------------------------------------------------- */

int or_lu(int n, const double *d, const double *e, double sigma, double pivthr,
          double *u1, double *u2, double *u3, double *l, unsigned char *swp)
{
    int replaced = 0;                        /* pivots moved to +-pivthr */
    double alpha = d[0] - sigma;             /* active row, column i     */
    double beta = n > 1 ? e[0] : 0.0;        /* active row, column i + 1 */
    for (int i = 0; i < n - 1; i++) {
        double b = e[i];                                  /* row i+1, col i   */
        double a1 = d[i + 1] - sigma;                     /* row i+1, col i+1 */
        double b1 = (i + 1 < n - 1) ? e[i + 1] : 0.0;     /* row i+1, col i+2 */
        if (fabs(alpha) >= fabs(b)) {
            double piv = alpha;
            if (fabs(piv) < pivthr) { piv = piv < 0.0 ? -pivthr : pivthr; replaced++; }
            u1[i] = piv; u2[i] = beta; u3[i] = 0.0; swp[i] = 0;
            l[i] = b / piv;
            alpha = a1 - l[i] * beta;
            beta = b1;
        } else {
            double piv = b;
            if (fabs(piv) < pivthr) { piv = piv < 0.0 ? -pivthr : pivthr; replaced++; }
            u1[i] = piv; u2[i] = a1; u3[i] = b1; swp[i] = 1;
            l[i] = alpha / piv;
            alpha = beta - l[i] * a1;
            beta = -(l[i] * b1);
        }
    }
    double piv = alpha;
    if (fabs(piv) < pivthr) { piv = piv < 0.0 ? -pivthr : pivthr; replaced++; }
    u1[n - 1] = piv; u2[n - 1] = 0.0; u3[n - 1] = 0.0; l[n - 1] = 0.0; swp[n - 1] = 0;
    return replaced;
}

/* x = U^{-1} L^{-1} P b, in place in b.  y is n doubles of scratch. */
void or_lu_solve(int n, const double *u1, const double *u2, const double *u3,
                 const double *l, const unsigned char *swp, double *b, double *y)
{
    double cur = b[0];
    for (int i = 0; i < n - 1; i++) {
        if (!swp[i]) { y[i] = cur; cur = b[i + 1] - l[i] * cur; }
        else         { y[i] = b[i + 1]; cur = cur - l[i] * b[i + 1]; }
    }
    y[n - 1] = cur;
    b[n - 1] = y[n - 1] / u1[n - 1];
    if (n > 1) b[n - 2] = (y[n - 2] - u2[n - 2] * b[n - 1]) / u1[n - 2];
    for (int i = n - 3; i >= 0; i--)
        b[i] = ((y[i] - u2[i] * b[i + 1]) - u3[i] * b[i + 2]) / u1[i];
}

/* ------------------------------------------------------------------------- */
/* Small dense helpers (plain loops).                                          */
/* ------------------------------------------------------------------------- */

static double nrm2(int n, const double *x)
{
    double s = 0.0;
    for (int i = 0; i < n; i++) s = s + x[i] * x[i];
    return sqrt(s);
}

static double sgn(double a) { return a >= 0.0 ? 1.0 : -1.0; }   /* sgn(0) = +1 */

/* ------------------------------------------------------------------------- */
/* Orthogonalization of one incoming vector against the reflectors of the     */
/* previous c vectors.  Y is n x M column-major (ld ldy), T is M x M          */
/* column-major upper triangular (ld ldt).  On entry v holds v_j; on exit it  */
/* holds q_j and column c of Y, T (the paper's index j = c + 1) is (re)set.   */
/* ------------------------------------------------------------------------- */

/* Householder vector of u (rows c..n-1 meaningful) as in Eq. (yt):
 * c_j = -sgn(u_jj) ||u_{j:n}||, y = [0; u_jj - c_j; u_{j+1:n}].
 * Reading for ||u_{j:n}|| = 0 (the paper is silent): H = I, i.e. y = 0, t = 0;
 * *brk is set to 1 in that case (the breakdown of the reflector), else 0.
 * Writes column c of Y; returns c_j and (through uj) u_jj. */
static double house_vec(int n, int c, const double *u, double *ycol, double *uj, int *brk)
{
    double alpha = u[c];
    double beta = nrm2(n - c, u + c);
    double gamma = -sgn(alpha) * beta;
    for (int i = 0; i < c; i++) ycol[i] = 0.0;
    if (beta == 0.0) {
        for (int i = c; i < n; i++) ycol[i] = 0.0;
    } else {
        for (int i = c; i < n; i++) ycol[i] = u[i];
        ycol[c] = alpha - gamma;
    }
    *uj = alpha;
    *brk = beta == 0.0;
    return gamma;
}

/* The compact-WY step in the reduced form of section 3.3.2, for member c
 * (the paper's j = c + 1) against the reflectors of members 0..c-1.
 *
 * Y_c = [L; Yhat] splits at row c: L holds rows 0..c-1 (lower triangular with
 * its diagonal), Yhat rows c..n-1; T_c is upper triangular.  Because every
 * y_l is zero above row l, only the rows of Q_c^T v at and below c are needed
 * to build the next reflector, and they are
 *     u_hat = v_hat - Yhat T_c^T (L^T v_top + Yhat^T v_hat),
 * with v_top, v_hat the rows of v above and from row c.  Eq. (yt) turns
 * u_hat into y_c and t_c = 1/(c_j^2 - u_jj c_j).  The new column of T is
 * -t_c T_c (Y_c^T y_c) = -t_c T_c (Yhat^T y_hat): the L rows of Y_c^T y_c
 * meet the zero top of y_c.  The iterate is replaced by
 *     q = (Y_{c+1} T_{c+1} Y_{c+1}^T - I) e_c = Y_{c+1} (T_{c+1} r) - e_c,
 * r = row c of Y_{c+1}.  The section prints this product with T^T; the form
 * of Eq. (cwy2) (and of Alg. 3) has T, which is what is used here.
 * Returns 1 when the reflector breaks down (||u_hat|| = 0), else 0. */
static int orth_cwy_new(int n, int c, double *Y, int ldy, double *T, int ldt, double *v,
                        double *w)
{
    double *x = w;              /* c: Y_c^T v, then T_c^T of it          */
    double *tmp = w + n;        /* c + 1                                  */
    double *uh = w + 2 * n;     /* rows c..n-1: u_hat                     */
    double *xr = w + 3 * n;     /* c + 1: T_{c+1} r                       */
    double *q = w + 4 * n;      /* n                                      */

    /* x_l = (Yhat^T v_hat)_l + (L^T v_top)_l, the L part summed first */
    for (int l = 0; l < c; l++) {
        double top = 0.0;
        for (int i = l; i < c; i++) top = top + Y[i + (size_t)l * ldy] * v[i];
        double bot = 0.0;
        for (int i = c; i < n; i++) bot = bot + Y[i + (size_t)l * ldy] * v[i];
        x[l] = bot + top;
    }
    /* x <- T_c^T x */
    for (int l = 0; l < c; l++) {
        double s = 0.0;
        for (int p = 0; p <= l; p++) s = s + T[p + (size_t)l * ldt] * x[p];
        tmp[l] = s;
    }
    for (int l = 0; l < c; l++) x[l] = tmp[l];
    /* u_hat = v_hat - Yhat x */
    for (int i = c; i < n; i++) {
        double s = 0.0;
        for (int l = 0; l < c; l++) s = s + Y[i + (size_t)l * ldy] * x[l];
        uh[i] = v[i] - s;
    }
    /* Eq. (yt): y_c (column c of Y) and t_c */
    double *ycol = Y + (size_t)c * ldy;
    double ujj;
    int brk;
    double gamma = house_vec(n, c, uh, ycol, &ujj, &brk);
    double tc = gamma == 0.0 ? 0.0 : 1.0 / (gamma * gamma - ujj * gamma);
    /* column c of T: -t_c T_c (Yhat^T y_hat), diagonal t_c */
    for (int l = 0; l < c; l++) {
        double s = 0.0;
        for (int i = c; i < n; i++) s = s + Y[i + (size_t)l * ldy] * ycol[i];
        tmp[l] = (-tc) * s;
    }
    for (int p = 0; p < c; p++) {
        double s = 0.0;
        for (int l = p; l < c; l++) s = s + T[p + (size_t)l * ldt] * tmp[l];
        T[p + (size_t)c * ldt] = s;
    }
    T[c + (size_t)c * ldt] = tc;
    /* xr = T_{c+1} r with r = row c of Y_{c+1} */
#ifdef OR_PRINTED_TRANSPOSE
    /* Test-only planted mistake: the transposed product as printed. */
    for (int l = 0; l <= c; l++) {
        double s = 0.0;
        for (int p = 0; p <= l; p++) s = s + T[p + (size_t)l * ldt] * Y[c + (size_t)p * ldy];
        xr[l] = s;
    }
#else
    for (int p = 0; p <= c; p++) {
        double s = 0.0;
        for (int l = p; l <= c; l++) s = s + T[p + (size_t)l * ldt] * Y[c + (size_t)l * ldy];
        xr[p] = s;
    }
#endif
    /* q = Y_{c+1} xr - e_c (row i of Y_{c+1} has nonzeros in columns 0..min(i, c)) */
    for (int i = 0; i < n; i++) {
        int lmax = i < c ? i : c;
        double s = 0.0;
        for (int l = 0; l <= lmax; l++) s = s + Y[i + (size_t)l * ldy] * xr[l];
        q[i] = s;
    }
    q[c] = q[c] - 1.0;
    for (int i = 0; i < n; i++) v[i] = q[i];
    return brk;
}

/* Ordinary implementation, section 3.3.1: full-length u_j = v_j - Y T^T Y^T v_j,
 * t_j = 2 / ||y_j||^2, t_hat = T (-t_j Y^T y_j), q_j = e_j - Y_j T_j Y_j^T e_j
 * (again T_j where the section prints T_j^T). */
static int orth_cwy_ordinary(int n, int c, double *Y, int ldy, double *T, int ldt, double *v,
                             double *w)
{
    double *vp = w;            /* c + 1 */
    double *tmp = w + n;       /* c + 1 */
    double *u = w + 2 * n;     /* n     */
    double *q = w + 4 * n;     /* n     */
    for (int i = 0; i < n; i++) u[i] = v[i];                       /* DCOPY */
    for (int l = 0; l < c; l++) {                                  /* DGEMV */
        double s = 0.0;
        for (int i = 0; i < n; i++) s = s + Y[i + (size_t)l * ldy] * u[i];
        vp[l] = s;
    }
    for (int l = 0; l < c; l++) {                                  /* DTRMV T^T */
        double s = 0.0;
        for (int p = 0; p <= l; p++) s = s + T[p + (size_t)l * ldt] * vp[p];
        tmp[l] = s;
    }
    for (int i = 0; i < n; i++) {                                  /* DGEMV */
        double s = 0.0;
        for (int l = 0; l < c; l++) s = s + Y[i + (size_t)l * ldy] * tmp[l];
        u[i] = u[i] - s;
    }
    double *ycol = Y + (size_t)c * ldy;
    double ujj;
    int brk;
    house_vec(n, c, u, ycol, &ujj, &brk);
    double ny = nrm2(n, ycol);
    double tj = ny == 0.0 ? 0.0 : 2.0 / (ny * ny);
    for (int l = 0; l < c; l++) {                                  /* DGEMV */
        double s = 0.0;
        for (int i = 0; i < n; i++) s = s + Y[i + (size_t)l * ldy] * ycol[i];
        tmp[l] = (-tj) * s;
    }
    for (int p = 0; p < c; p++) {                                  /* DTRMV T */
        double s = 0.0;
        for (int l = p; l < c; l++) s = s + T[p + (size_t)l * ldt] * tmp[l];
        T[p + (size_t)c * ldt] = s;
    }
    T[c + (size_t)c * ldt] = tj;
    for (int l = 0; l <= c; l++) vp[l] = Y[c + (size_t)l * ldy];   /* DCOPY row j */
    for (int p = 0; p <= c; p++) {                                 /* DTRMV T_j */
        double s = 0.0;
        for (int l = p; l <= c; l++) s = s + T[p + (size_t)l * ldt] * vp[l];
        tmp[p] = s;
    }
    for (int i = 0; i < n; i++) q[i] = (i == c) ? 1.0 : 0.0;       /* DCOPY e_j */
    for (int i = 0; i < n; i++) {                                  /* DGEMV */
        double s = 0.0;
        for (int l = 0; l <= c; l++) s = s + Y[i + (size_t)l * ldy] * tmp[l];
        q[i] = q[i] - s;
    }
    for (int i = 0; i < n; i++) v[i] = q[i];
    return brk;
}

/* Householder orthogonalization, Alg. 2: apply H_1 .. H_{j-1} one at a time,
 * form y_j, t_j = 2/||y_j||^2 from u_j, then q_j = H_1 ... H_j e_j.  Only the
 * reflector vectors (columns of Y) and their t (diagonal of T) are used. */
static int orth_householder(int n, int c, double *Y, int ldy, double *T, int ldt, double *v,
                            double *w)
{
    double *u = w + 2 * n;
    double *q = w + 4 * n;
    for (int i = 0; i < n; i++) u[i] = v[i];
    for (int r = 0; r < c; r++) {
        const double *y = Y + (size_t)r * ldy;
        double t = T[r + (size_t)r * ldt];
        double s = 0.0;
        for (int i = 0; i < n; i++) s = s + y[i] * u[i];
        for (int i = 0; i < n; i++) u[i] = u[i] - (t * s) * y[i];
    }
    double *ycol = Y + (size_t)c * ldy;
    double ujj;
    int brk;
    house_vec(n, c, u, ycol, &ujj, &brk);
    double ny = nrm2(n, ycol);
    double tj = ny == 0.0 ? 0.0 : 2.0 / (ny * ny);
    T[c + (size_t)c * ldt] = tj;
    for (int i = 0; i < n; i++) q[i] = (i == c) ? 1.0 : 0.0;
    for (int r = c; r >= 0; r--) {
        const double *y = Y + (size_t)r * ldy;
        double t = T[r + (size_t)r * ldt];
        double s = 0.0;
        for (int i = 0; i < n; i++) s = s + y[i] * q[i];
        for (int i = 0; i < n; i++) q[i] = q[i] - (t * s) * y[i];
    }
    for (int i = 0; i < n; i++) v[i] = q[i];
    return brk;
}

enum { OR_CWY_NEW = 0, OR_CWY_ORDINARY = 1, OR_HOUSEHOLDER = 2, OR_MGS = 3 };

/* The stop test of the repeat loop (Alg. 1 and Alg. 4 repeat "until some
 * condition is met" and leave the condition open).  Default reading: a fixed
 * number of iterations.  The growth rule (iters = OR_STOP_GROWTH), in the
 * manner of the inverse-iteration code the paper starts from: a solve
 * (T - lambda I) x = v with ||v||_2 = 1 has converged when its growth is large,
 * ||x||_2 >= 1 / (n eps ||T||_1) -- 1/||x||_2 is the residual of x/||x||_2 --
 * with ||x||_2^2 summed from the last row up with fused multiply-adds; after
 * the first converged solve the vector gets OR_STOP_EXTRA more iterations, at
 * most OR_STOP_MAXITS in all. */
enum { OR_STOP_GROWTH = -1, OR_STOP_EXTRA = 2, OR_STOP_MAXITS = 5 };

static int or_solve_converged(int n, const double *x, double gtau)
{
    double ss = 0.0;
    for (int i = n - 1; i >= 0; i--) ss = fma(x[i], x[i], ss);
    return sqrt(ss) * gtau >= 1.0;
}

/* Per-vector status bits of or_eigvecs: a non-finite entry in the output; a
 * reflector of one of its orthogonalizations broke down (||u_hat|| = 0, so
 * H = I); a pivot of its shifted LU fell below eps ||T||_1 and was replaced;
 * under the growth rule, no solve of the vector converged. */
enum { OR_ST_NONFINITE = 1, OR_ST_BREAKDOWN = 2, OR_ST_PIVOT = 4, OR_ST_NOCONV = 8 };

/* Householder vector and t of the first vector of a sequence (Alg. 3 line 1). */
static void orth_first(int n, int variant, double *Y, int ldy, double *T, int ldt,
                       const double *u)
{
    double ujj;
    int brk;
    double gamma = house_vec(n, 0, u, Y, &ujj, &brk);
    double tj;
    if (variant == OR_CWY_NEW) {
        tj = gamma == 0.0 ? 0.0 : 1.0 / (gamma * gamma - ujj * gamma);
    } else {
        double ny = nrm2(n, Y);
        tj = ny == 0.0 ? 0.0 : 2.0 / (ny * ny);
    }
    T[0] = tj;
    (void)ldy; (void)ldt;
}

/* Incremental orthogonalization of the columns of V (section 3, all vectors
 * given in advance): Q[:, j] from V[:, 0..j].  Y (n x m) and T (m x m) receive
 * the compact-WY factors for the cWY variants (only diag(T) for Householder).
 * variant: 0 new cWY (3.3.2), 1 ordinary cWY (3.3.1), 2 Householder (Alg. 2),
 * 3 MGS.  brk (may be NULL, m entries) receives 1 for a column whose reflector
 * broke down (||u_hat|| = 0; Householder variants only), else 0. */
int or_orthogonalize(int n, int m, const double *V, int ldv, double *Q, int ldq,
                     double *Y, double *T, int variant, int *brk)
{
    if (n < 1 || m < 1 || m > n) return -1;
    double *w = (double *)calloc((size_t)5 * n + 8, sizeof(double));
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    if (!w || !v) { free(w); free(v); return -2; }
    memset(Y, 0, sizeof(double) * (size_t)n * m);
    memset(T, 0, sizeof(double) * (size_t)m * m);
    for (int j = 0; j < m; j++) {
        for (int i = 0; i < n; i++) v[i] = V[i + (size_t)j * ldv];
        if (brk) brk[j] = 0;
        if (variant == OR_MGS) {
            for (int r = 0; r < j; r++) {
                double s = 0.0;
                for (int i = 0; i < n; i++) s = s + v[i] * Q[i + (size_t)r * ldq];
                for (int i = 0; i < n; i++) v[i] = v[i] - s * Q[i + (size_t)r * ldq];
            }
            double nv = nrm2(n, v);
            for (int i = 0; i < n; i++) Q[i + (size_t)j * ldq] = v[i] / nv;
            continue;
        }
        if (j == 0) {
            /* first step of Alg. 3: y_1, t_1 from u_1 = v_1, q_1 = (I - Y_1 T_1 Y_1^T) e_1 */
            orth_first(n, variant, Y, n, T, m, v);
            double t = T[0];
            for (int i = 0; i < n; i++) Q[i] = -(t * Y[0]) * Y[i];
            Q[0] = Q[0] + 1.0;
            if (variant == OR_CWY_NEW)              /* section 3.3.2 sign of q_j */
                for (int i = 0; i < n; i++) Q[i] = -Q[i];
            continue;
        }
        int b;
        if (variant == OR_CWY_NEW) b = orth_cwy_new(n, j, Y, n, T, m, v, w);
        else if (variant == OR_CWY_ORDINARY) b = orth_cwy_ordinary(n, j, Y, n, T, m, v, w);
        else b = orth_householder(n, j, Y, n, T, m, v, w);
        if (brk) brk[j] = b;
        for (int i = 0; i < n; i++) Q[i + (size_t)j * ldq] = v[i];
    }
    free(w);
    free(v);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Inverse iteration, Alg. 4 (compact WY) and Alg. 1 (MGS).                    */
/* ------------------------------------------------------------------------- */

/* Computes eigenvectors Z[:, j] (column-major, ld ldz) of T = tridiag(e, d, e)
 * for the m eigenvalues W[0..m-1] (ascending).  If Win is NULL they are the
 * bisection eigenvalues il..iu and are written to W; otherwise W = Win and
 * il is only the base of the start-vector key (eigenvalue j uses key index
 * il + j).  orth: 0 new cWY (Alg. 4 with section 3.3.2), 1 ordinary cWY,
 * 2 Householder, 3 MGS (Alg. 1).  iters: fixed iteration count (the paper
 * leaves the stop test of the repeat loop open; it is read as a fixed count),
 * or OR_STOP_GROWTH for the growth rule above.  Each output
 * column is normalized to unit 2-norm and its largest-magnitude entry (lowest
 * index on ties) made positive.  status (may be NULL, m entries) receives the
 * OR_ST_* bits of each vector.  Returns the number of clusters, or < 0. */
int or_eigvecs(int n, const double *d, const double *e, int il, int iu, const double *Win,
               int orth, int iters, uint64_t seed, double *W, double *Z, int ldz, int *status)
{
    if (n < 1 || il < 1 || iu < il || ldz < n) return -1;
    if (!Win && iu > n) return -1;
    int m = iu - il + 1;
    if (m > n) return -1;
    or_params p;
    if (or_setup(n, d, e, &p)) return -2;
    if (Win) { for (int j = 0; j < m; j++) W[j] = Win[j]; }
    else if (or_bisect(n, d, e, il, iu, W)) return -2;

    int *cst = (int *)malloc(sizeof(int) * (size_t)m);
    int *csz = (int *)malloc(sizeof(int) * (size_t)m);
    double *u1 = (double *)malloc(sizeof(double) * (size_t)n * 5);
    unsigned char *swp = (unsigned char *)malloc((size_t)n);
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)calloc((size_t)5 * n + 8, sizeof(double));
    if (!cst || !csz || !u1 || !swp || !v || !y || !w) return -2;
    double *u2 = u1 + n, *u3 = u1 + 2 * (size_t)n, *lm = u1 + 3 * (size_t)n;
    int ncl = or_clusters(m, W, p.tol, cst, csz);
    double gtau = ((double)n * DBL_EPSILON) * p.norm1;   /* growth rule threshold */

    int maxsz = 1;
    for (int c = 0; c < ncl; c++) if (csz[c] > maxsz) maxsz = csz[c];
    double *Y = (double *)calloc((size_t)n * maxsz, sizeof(double));
    double *T = (double *)calloc((size_t)maxsz * maxsz, sizeof(double));
    if (!Y || !T) return -2;

    for (int cl = 0; cl < ncl; cl++) {
        int j1 = cst[cl];
        for (int j = j1; j < j1 + csz[cl]; j++) {
            int jc = j - j1;                     /* position in the cluster */
            int st = 0;
            if (or_lu(n, d, e, W[j], p.pivthr, u1, u2, u3, lm, swp) > 0) st |= OR_ST_PIVOT;
            or_start_vector(seed, (int64_t)il + j, n, v);
            int kend = iters > 0 ? iters : OR_STOP_MAXITS;
            int conv = 0;
            for (int k = 1; k <= kend; k++) {
                double nv = nrm2(n, v);          /* normalize v^(k-1) */
                for (int i = 0; i < n; i++) v[i] = v[i] / nv;
                or_lu_solve(n, u1, u2, u3, lm, swp, v, y);   /* Eq. (1) */
                if (iters < 0 && !conv && or_solve_converged(n, v, gtau)) {
                    conv = 1;
                    if (k + OR_STOP_EXTRA < kend) kend = k + OR_STOP_EXTRA;
                }
                if (jc == 0) continue;
                if (orth == OR_MGS) {            /* Alg. 1: MGS against v_{j1}..v_{j-1} */
                    for (int r = j1; r < j; r++) {
                        const double *zr = Z + (size_t)r * ldz;
                        double s = 0.0;
                        for (int i = 0; i < n; i++) s = s + v[i] * zr[i];
                        for (int i = 0; i < n; i++) v[i] = v[i] - s * zr[i];
                    }
                    continue;
                }
                if (jc == 1 && k == 1)           /* Alg. 4: Y_1, T_1 from v_{j1} */
                    orth_first(n, orth, Y, n, T, maxsz, Z + (size_t)j1 * ldz);
                int b;
                if (orth == OR_CWY_NEW) b = orth_cwy_new(n, jc, Y, n, T, maxsz, v, w);
                else if (orth == OR_CWY_ORDINARY) b = orth_cwy_ordinary(n, jc, Y, n, T, maxsz, v, w);
                else b = orth_householder(n, jc, Y, n, T, maxsz, v, w);
                if (b) st |= OR_ST_BREAKDOWN;
            }
            if (iters < 0 && !conv) st |= OR_ST_NOCONV;
            double nv = nrm2(n, v);              /* normalize v^(k) to v_j */
            double *z = Z + (size_t)j * ldz;
            for (int i = 0; i < n; i++) z[i] = v[i] / nv;
            for (int i = 0; i < n; i++) if (!isfinite(z[i])) { st |= OR_ST_NONFINITE; break; }
            if (status) status[j] = st;
        }
    }
    /* Output sign: largest-magnitude entry positive (lowest index on ties).
     * Applied after all clusters so that Y_1 is built from the unflipped
     * normalized vector, as the GPU library does. */
    for (int j = 0; j < m; j++) {
        double *z = Z + (size_t)j * ldz;
        int im = 0;
        for (int i = 1; i < n; i++) if (fabs(z[i]) > fabs(z[im])) im = i;
        if (z[im] < 0.0) for (int i = 0; i < n; i++) z[i] = -z[i];
    }
    free(cst); free(csz); free(u1); free(swp); free(v); free(y); free(w); free(Y); free(T);
    return ncl;
}

/* ------------------------------------------------------------------------- */
/* Splitting into unreduced blocks.  The paper does not split; the LAPACK     */
/* bisection and inverse-iteration codes its method builds on (section 4,     */
/* section 5.1) work block by block.  Reading: e_i is negligible when         */
/*     e_i^2 <= eps^2 |d_i d_{i+1}| + DBL_MIN,                                 */
/* and T is then the direct sum of its unreduced blocks, each solved as an    */
/* independent problem (its own norm, cluster gap and pivot floor).  The      */
/* eigenvalues of all blocks, in ascending order with ties taken lower block  */
/* first, are numbered 1..n; il..iu select from that order.  Eigenvalue l     */
/* (0-based, ascending) of the block that starts at row s uses start-vector   */
/* key s + 1 + l, rows numbered within the block; its eigenvector is the      */
/* block's, zero outside the block.                                           */
/* ------------------------------------------------------------------------- */

/* Block starts: bstart[0] = 0 < bstart[1] < ... < bstart[nb] = n.  Returns nb. */
int or_split_points(int n, const double *d, const double *e, int *bstart)
{
    int nb = 0;
    bstart[nb++] = 0;
    for (int i = 0; i < n - 1; i++) {
        double lim = (DBL_EPSILON * DBL_EPSILON) * fabs(d[i] * d[i + 1]) + DBL_MIN;
        if (e[i] * e[i] <= lim) bstart[nb++] = i + 1;
    }
    bstart[nb] = n;
    return nb;
}

typedef struct { double v; int b, l; } or_bval;

static int bval_cmp(const void *pa, const void *pb)
{
    const or_bval *a = (const or_bval *)pa, *b = (const or_bval *)pb;
    if (a->v < b->v) return -1;
    if (a->v > b->v) return 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    return a->l < b->l ? -1 : (a->l > b->l);
}

/* As or_eigvecs (computed eigenvalues il..iu) on the split matrix.  blk (may
 * be NULL, m entries) receives the block index of each output column.
 * Returns the number of blocks, or < 0. */
int or_eigvecs_split(int n, const double *d, const double *e, int il, int iu, int orth,
                     int iters, uint64_t seed, double *W, double *Z, int ldz, int *status,
                     int *blk)
{
    if (n < 1 || il < 1 || iu < il || iu > n || ldz < n) return -1;
    int m = iu - il + 1;
    int *bs = (int *)malloc(sizeof(int) * (size_t)(n + 1));
    double *vals = (double *)malloc(sizeof(double) * (size_t)n);
    or_bval *all = (or_bval *)malloc(sizeof(or_bval) * (size_t)n);
    int *pos = (int *)malloc(sizeof(int) * (size_t)n);   /* output column of (block row s + l) */
    if (!bs || !vals || !all || !pos) return -2;
    int nb = or_split_points(n, d, e, bs);
    for (int b = 0; b < nb; b++) {
        int s = bs[b], nbk = bs[b + 1] - bs[b];
        if (or_bisect(nbk, d + s, e + s, 1, nbk, vals + s)) return -2;
        for (int l = 0; l < nbk; l++) { all[s + l].v = vals[s + l]; all[s + l].b = b; all[s + l].l = l; }
    }
    qsort(all, (size_t)n, sizeof(or_bval), bval_cmp);
    for (int k = 0; k < n; k++) pos[bs[all[k].b] + all[k].l] = k - (il - 1);
    for (int j = 0; j < m; j++)
        for (int i = 0; i < n; i++) Z[i + (size_t)j * ldz] = 0.0;
    for (int b = 0; b < nb; b++) {
        int s = bs[b], nbk = bs[b + 1] - bs[b];
        int lo = -1, hi = -2;                     /* selected local indices: a range */
        for (int l = 0; l < nbk; l++) {
            int p = pos[s + l];
            if (p >= 0 && p < m) { if (lo < 0) lo = l; hi = l; }
        }
        if (lo < 0) continue;
        int mb = hi - lo + 1;
        double *Wb = (double *)malloc(sizeof(double) * (size_t)mb);
        double *Zb = (double *)malloc(sizeof(double) * (size_t)nbk * mb);
        int *stb = (int *)malloc(sizeof(int) * (size_t)mb);
        if (!Wb || !Zb || !stb) return -2;
        if (or_eigvecs(nbk, d + s, e + s, s + 1 + lo, s + 1 + hi, vals + s + lo, orth, iters,
                       seed, Wb, Zb, nbk, stb) < 0) return -2;
        for (int j = 0; j < mb; j++) {
            int p = pos[s + lo + j];
            W[p] = Wb[j];
            for (int i = 0; i < nbk; i++) Z[(s + i) + (size_t)p * ldz] = Zb[i + (size_t)j * nbk];
            if (status) status[p] = stb[j];
            if (blk) blk[p] = b;
        }
        free(Wb); free(Zb); free(stb);
    }
    free(bs); free(vals); free(all); free(pos);
    return nb;
}

/* ------------------------------------------------------------------------- */
/* Singular vectors of a bidiagonal matrix, the application the paper names   */
/* as future work (section 6), through the Golub-Kahan tridiagonal: for upper */
/* bidiagonal B (diagonal a[0..n-1], superdiagonal b[0..n-2]), the symmetric  */
/* tridiagonal of order 2n with zero diagonal and off-diagonal                */
/* (a_0, b_0, a_1, b_1, ..., b_{n-2}, a_{n-1}) has eigenvalues +-sigma_i, and */
/* an eigenvector (x_0, y_0, x_1, y_1, ...) of +sigma gives B x = sigma y and */
/* B^T y = sigma x.  Singular values in ascending order, indices il..iu of    */
/* 1..n, are the tridiagonal's eigenvalues n + il .. n + iu (the method with  */
/* its clusters formed among those, start-vector keys n + il + j); V takes    */
/* the x half and U the y half of each vector, each normalized to unit        */
/* 2-norm (reading: the halves are normalized separately).                    */
/* ------------------------------------------------------------------------- */

int or_bidiag_svd(int n, const double *a, const double *b, int il, int iu, int orth, int iters,
                  uint64_t seed, double *S, double *U, int ldu, double *V, int ldv, int *status)
{
    if (n < 1 || il < 1 || iu < il || iu > n || ldu < n || ldv < n) return -1;
    int N = 2 * n, m = iu - il + 1;
    double *dg = (double *)calloc((size_t)N, sizeof(double));
    double *eg = (double *)malloc(sizeof(double) * (size_t)(N - 1));
    double *Zg = (double *)malloc(sizeof(double) * (size_t)N * m);
    if (!dg || !eg || !Zg) return -2;
    for (int k = 0; k < n; k++) {
        eg[2 * k] = a[k];
        if (k < n - 1) eg[2 * k + 1] = b[k];
    }
    int ncl = or_eigvecs(N, dg, eg, n + il, n + iu, NULL, orth, iters, seed, S, Zg, N, status);
    if (ncl < 0) return ncl;
    for (int j = 0; j < m; j++) {
        const double *z = Zg + (size_t)j * N;
        double sx = 0.0, sy = 0.0;
        for (int k = 0; k < n; k++) { sx = sx + z[2 * k] * z[2 * k]; sy = sy + z[2 * k + 1] * z[2 * k + 1]; }
        double nx = sqrt(sx), ny = sqrt(sy);
        for (int k = 0; k < n; k++) {
            V[k + (size_t)j * ldv] = z[2 * k] / nx;
            U[k + (size_t)j * ldu] = z[2 * k + 1] / ny;
        }
    }
    free(dg); free(eg); free(Zg);
    return ncl;
}
