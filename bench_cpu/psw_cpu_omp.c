/*
 * psw_cpu_omp.c -- the decomposed sweep on all host cores (OpenMP over
 * subdomains), the CPU baseline that the benchmark reports beside the
 * single-threaded oracle.  It is the shared-memory use of the method that
 * the paper points out (Sec. 3: subdomains are swept independently, no
 * message passing is needed): given the old iterate, every subdomain
 * computes its own points, and recomputes the partner points across its
 * coupled start faces (the 2x2 / 4x4 / 8x8 blocks of eqs. 1d:sorc,
 * 2d:sor2b2, 2d:sor4b4 and Sec. 4) instead of exchanging them.
 *
 * It is neither the GPU path nor the oracle: tests/test_cpu_parallel.py holds
 * it to the oracle.  Build: gcc -O3 -fopenmp -shared -fPIC.
 *
 * One sweep solves, for every point X of subdomain s,
 *   Piv_X u_X - sum_{Y upstream of X} a_XY u_Y = f_X + [uold: (Piv_X - a^P_X) uold_X
 *                                                         + sum_{Y downstream} a_XY uold_Y]
 * with Piv = a^P / w (w of the start corner of X's subdomain) for the
 * stationary sweep (uold given), or Piv = piv (given) and no old iterate for
 * a start-coupled preconditioner half-sweep.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t idx3(const int64_t n[3], int64_t x, int64_t y, int64_t z) { return x + n[0] * (y + n[1] * z); }
static inline int dkk(int a, int s) { return s < 0 ? 1 + 2 * a : 2 + 2 * a; }

/* contiguous ranges, the first n mod p one point longer */
static void range_of(int64_t n, int p, int r, int64_t *lo, int64_t *len)
{
    int64_t base = n / p, rem = n % p;
    *len = base + (r < rem ? 1 : 0);
    *lo = r * base + (r < rem ? r : rem);
}

/* small dense solve with partial pivoting */
static void solve_small(int m, double A[8][8], double *b)
{
    for (int k = 0; k < m; ++k) {
        int piv = k;
        for (int i = k + 1; i < m; ++i)
            if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
        if (piv != k) {
            for (int j = 0; j < m; ++j) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int i = k + 1; i < m; ++i) {
            double l = A[i][k] / A[k][k];
            for (int j = k; j < m; ++j) A[i][j] -= l * A[k][j];
            b[i] -= l * b[k];
        }
    }
    for (int i = m - 1; i >= 0; --i) {
        double acc = b[i];
        for (int j = i + 1; j < m; ++j) acc -= A[i][j] * b[j];
        b[i] = acc / A[i][i];
    }
}

/*
 * dim 1..3, n[3] (1 on unused axes), p[3], dirs[3*nsub] (subdomain s = r + p0 (q + p1 t)),
 * diag[2*dim+1], omega8 (by start corner; stationary only), piv (preconditioner only, else NULL),
 * uold (stationary, else NULL), f, out.  Returns 0, or -1 on bad arguments / -2 on memory.
 */
int cpu_dsweep(int dim, const int64_t n_in[3], const int p_in[3], const int8_t *dirs, const double *const *diag,
               const double *omega8, const double *piv, const double *uold, const double *f, double *out)
{
    int64_t n[3] = {1, 1, 1};
    int p[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) { n[a] = n_in[a]; p[a] = p_in[a]; }
    const int nsub = p[0] * p[1] * p[2];
    int err = 0;
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int s = 0; s < nsub; ++s) {
        const int sc[3] = {s % p[0], (s / p[0]) % p[1], s / (p[0] * p[1])};
        int64_t lo[3], len[3];
        int d[3], cpl[3];
        for (int a = 0; a < 3; ++a) {
            range_of(n[a], p[a], sc[a], &lo[a], &len[a]);
            d[a] = a < dim ? dirs[3 * s + a] : 1;
            /* the start side of axis a has a neighbour subdomain: it starts there too (neighbours
               sweep in opposite directions), so the face is coupled */
            cpl[a] = a < dim && (d[a] > 0 ? lo[a] > 0 : lo[a] + len[a] < n[a]);
        }
        /* extended box in local sweep coordinates: l_a from -cpl[a] to len[a]-1 */
        int64_t ext[3], cnt = 1;
        for (int a = 0; a < 3; ++a) { ext[a] = len[a] + cpl[a]; cnt *= ext[a]; }
        double *w = (double *)malloc(sizeof(double) * cnt);
        if (!w) { err |= 1; continue; }
        /* global coordinate of local l on axis a */
#define GC(a, l) (d[a] > 0 ? lo[a] + (l) : lo[a] + len[a] - 1 - (l))
#define WI(l0, l1, l2) (((l0) + cpl[0]) + ext[0] * (((l1) + cpl[1]) + ext[1] * ((l2) + cpl[2])))
        for (int64_t l2 = 0; l2 < len[2]; ++l2)
            for (int64_t l1 = 0; l1 < len[1]; ++l1)
                for (int64_t l0 = 0; l0 < len[0]; ++l0) {
                    const int64_t l[3] = {l0, l1, l2};
                    int A[3], na = 0;
                    for (int a = 0; a < dim; ++a)
                        if (cpl[a] && l[a] == 0) A[na++] = a;
                    const int m = 1 << na;
                    double M[8][8], b[8];
                    int64_t bl[8][3];
                    for (int i = 0; i < m; ++i) {
                        for (int a = 0; a < 3; ++a) bl[i][a] = l[a];
                        for (int k = 0; k < na; ++k)
                            if (i & (1 << k)) bl[i][A[k]] = -1;
                    }
                    for (int i = 0; i < m; ++i) {
                        for (int j = 0; j < m; ++j) M[i][j] = 0.0;
                        const int64_t gx[3] = {GC(0, bl[i][0]), GC(1, bl[i][1]), GC(2, bl[i][2])};
                        const int64_t X = idx3(n, gx[0], gx[1], gx[2]);
                        /* the direction and start corner of X's own subdomain: flipped on the shifted axes */
                        int dx[3], corner = 0;
                        for (int a = 0; a < 3; ++a) {
                            dx[a] = bl[i][a] < 0 ? -d[a] : d[a];
                            if (a < dim && dx[a] < 0) corner |= 1 << a;
                        }
                        const double pX = piv ? piv[X] : diag[0][X] / omega8[corner];
                        M[i][i] = pX;
                        double r = f[X];
                        if (uold) r += (pX - diag[0][X]) * uold[X];
                        for (int a = 0; a < dim; ++a)
                            for (int sd = -1; sd <= 1; sd += 2) {
                                int64_t q[3] = {gx[0], gx[1], gx[2]};
                                q[a] += sd;
                                if (q[a] < 0 || q[a] >= n[a]) continue;
                                const double cf = diag[dkk(a, sd)][X];
                                const int64_t Q = idx3(n, q[0], q[1], q[2]);
                                if (sd == -dx[a]) {
                                    /* upstream: in the block, or computed earlier in the extended box */
                                    int64_t lq[3] = {bl[i][0], bl[i][1], bl[i][2]};
                                    lq[a] += bl[i][a] < 0 ? 1 : -1; /* towards the face / back along the sweep */
                                    if (bl[i][a] < 0) lq[a] = 0;
                                    int jb = -1;
                                    for (int j = 0; j < m; ++j)
                                        if (bl[j][0] == lq[0] && bl[j][1] == lq[1] && bl[j][2] == lq[2]) jb = j;
                                    if (jb >= 0) M[i][jb] -= cf;
                                    else r += cf * w[WI(lq[0], lq[1], lq[2])];
                                } else if (uold) {
                                    r += cf * uold[Q]; /* downstream: old value */
                                }
                            }
                        b[i] = r;
                    }
                    solve_small(m, M, b);
                    for (int i = 0; i < m; ++i) w[WI(bl[i][0], bl[i][1], bl[i][2])] = b[i];
                    out[idx3(n, GC(0, l0), GC(1, l1), GC(2, l2))] = b[0];
                }
#undef GC
#undef WI
        free(w);
    }
    return err ? -2 : 0;
}

int cpu_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* STREAM triad a = b + s c over n doubles, reps times; returns the best bytes/s */
double cpu_triad_bytes_per_s(int64_t n, int reps)
{
    double *a = (double *)malloc(sizeof(double) * n), *b = (double *)malloc(sizeof(double) * n),
           *c = (double *)malloc(sizeof(double) * n);
    if (!a || !b || !c) { free(a); free(b); free(c); return -1.0; }
#pragma omp parallel for
    for (int64_t i = 0; i < n; ++i) { a[i] = 0.0; b[i] = 1.0; c[i] = 2.0; }
    double best = 0.0;
    for (int r = 0; r < reps; ++r) {
#ifdef _OPENMP
        double t0 = omp_get_wtime();
#endif
#pragma omp parallel for
        for (int64_t i = 0; i < n; ++i) a[i] = b[i] + 3.0 * c[i];
#ifdef _OPENMP
        double dt = omp_get_wtime() - t0;
        if (dt > 0 && 24.0 * n / dt > best) best = 24.0 * n / dt;
#endif
    }
    free(a); free(b); free(c);
    return best;
}
