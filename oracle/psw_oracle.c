/*
 * psw_oracle.c -- plain, slow CPU FP64 oracle for the decomposed SOR / SSOR /
 * ILU(0) sweeps of R. Tavakoli, "Parallelizing sequential sweeping on
 * structured grids -- fully parallel SOR/ILU preconditioners for structured
 * n-diagonal matrices".
 *
 * TEST INFRASTRUCTURE.  This library exists to check the GPU library.  Only
 * the test suite, the package smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no source, header, table or helper with the
 * GPU path.  Build: gcc -O2 -ffp-contract=off -shared -fPIC (no intrinsics).
 *
 * Conventions (see the header of oracle.py for the full list of readings):
 *  - dim in {1,2,3}; n[a] interior points on axis a (1 for unused axes);
 *    point index P = x + n0*(y + n1*z) (x fastest).  Boundary points are not
 *    stored: Dirichlet data are folded into f (Sec. 2, eq. 1d:mat; Sec. 3).
 *  - diag[k], k = 0..2*dim: P, W, E, S, N, B, F.  Row P of A reads
 *      diag0[P] u_P - sum_{k>0} diag_k[P] u_{P+e_k} = f_P      (eq. d2d)
 *    and couplings that point outside the grid are ignored.
 *  - Subdomains: p[a] contiguous ranges per axis; the first n mod p ranges get
 *    ceil(n/p) points (Sec. 3: sub-domains of nearly equal size).  Subdomain id
 *    s = r + p0*(q + p1*t).
 *  - A direction is a sign per axis: +1 sweeps towards increasing index.
 *    Neighbour X of P is "upstream" when it lies on the side where the sweep
 *    of P's own subdomain begins.  Upstream values are new, downstream values
 *    are old (eqs. 1d:sorl/sorr, sor2d_sw..sor2d_nw).
 *  - Coupled blocks: a point on a start face of its subdomain whose
 *    neighbour across that face exists is solved jointly with the partner
 *    point(s) across every such face: 2x2 on faces (eq. 1d:sorc, eq.
 *    2d:sor2b2), 4x4 at 2D cross points and along 3D edges (eq. 2d:sor4b4),
 *    8x8 at 3D corners (Sec. 4).  Each block is solved by Gaussian
 *    elimination with partial pivoting, in rows scaled as in the paper
 *    (unit diagonal, -omega*a/a^P off the diagonal).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2
#define OR_EPIVOT -6
#define OR_ESINGULAR -9

typedef struct {
    int dim;
    int64_t n[3];
    int64_t N;
    int p[3];
    int nsub;
    int64_t *lo[3], *hi[3]; /* inclusive range bounds per axis */
    int *own[3];            /* coordinate -> range index per axis */
} grid_t;

/* ------------------------------------------------------------------ */
/* Partition: contiguous ranges, first n mod p ranges one point longer. */
int or_partition(int64_t n, int p, int64_t *lo, int64_t *hi)
{
    if (n < 1 || p < 1 || p > n) return OR_EINVAL;
    int64_t base = n / p, rem = n % p, start = 0;
    for (int r = 0; r < p; ++r) {
        int64_t len = base + (r < rem ? 1 : 0);
        lo[r] = start;
        hi[r] = start + len - 1;
        start += len;
    }
    return OR_OK;
}

static void grid_free(grid_t *g)
{
    for (int a = 0; a < 3; ++a) {
        free(g->lo[a]); free(g->hi[a]); free(g->own[a]);
        g->lo[a] = g->hi[a] = NULL; g->own[a] = NULL;
    }
}

static int grid_init(grid_t *g, int dim, const int64_t n[3], const int p[3])
{
    memset(g, 0, sizeof(*g));
    if (dim < 1 || dim > 3) return OR_EINVAL;
    g->dim = dim;
    g->N = 1;
    g->nsub = 1;
    for (int a = 0; a < 3; ++a) {
        g->n[a] = (a < dim) ? n[a] : 1;
        g->p[a] = (a < dim && p) ? p[a] : 1;
        if (g->n[a] < 1 || g->p[a] < 1 || g->p[a] > g->n[a]) { grid_free(g); return OR_EINVAL; }
        g->N *= g->n[a];
        g->nsub *= g->p[a];
        g->lo[a] = (int64_t *)malloc(sizeof(int64_t) * g->p[a]);
        g->hi[a] = (int64_t *)malloc(sizeof(int64_t) * g->p[a]);
        g->own[a] = (int *)malloc(sizeof(int) * g->n[a]);
        if (!g->lo[a] || !g->hi[a] || !g->own[a]) { grid_free(g); return OR_ENOMEM; }
        or_partition(g->n[a], g->p[a], g->lo[a], g->hi[a]);
        for (int r = 0; r < g->p[a]; ++r)
            for (int64_t c = g->lo[a][r]; c <= g->hi[a][r]; ++c) g->own[a][c] = r;
    }
    return OR_OK;
}

static inline void coords_of(const grid_t *g, int64_t P, int64_t c[3])
{
    c[0] = P % g->n[0];
    c[1] = (P / g->n[0]) % g->n[1];
    c[2] = P / (g->n[0] * g->n[1]);
}

static inline int64_t index_of(const grid_t *g, const int64_t c[3])
{
    return c[0] + g->n[0] * (c[1] + g->n[1] * c[2]);
}

static inline int sub_of(const grid_t *g, const int64_t c[3])
{
    return g->own[0][c[0]] + g->p[0] * (g->own[1][c[1]] + g->p[1] * g->own[2][c[2]]);
}

/* diagonal index for the coupling of a point to its neighbour on axis a,
   side s (-1: W/S/B, +1: E/N/F) */
static inline int dk(int a, int s) { return s < 0 ? 1 + 2 * a : 2 + 2 * a; }

/* ------------------------------------------------------------------ */
/* Direction schedule (Sec. 3, Sweeping directions; Sec. 4).
 * The base cycle sigma_k is used by subdomain (0,0,0); along each axis the
 * sign is flipped for odd subdomain coordinates, so neighbours always sweep
 * in opposite directions.  Consecutive pairs (sigma_{2i}, sigma_{2i+1}) are
 * mutually reversed; each pair uses a new diagonal.  phase=1 swaps the two
 * members of every pair. */
static const int SIG1[2][3] = {{+1, 1, 1}, {-1, 1, 1}};
static const int SIG2[4][3] = {{-1, -1, 1}, {+1, +1, 1}, {+1, -1, 1}, {-1, +1, 1}};
static const int SIG3[8][3] = {{-1, -1, -1}, {+1, +1, +1}, {+1, -1, -1}, {-1, +1, +1},
                               {-1, +1, -1}, {+1, -1, +1}, {+1, +1, -1}, {-1, -1, +1}};

int or_schedule(int dim, const int p[3], int64_t iter, int phase, int8_t *dirs)
{
    if (dim < 1 || dim > 3 || iter < 0) return OR_EINVAL;
    int period = 1 << dim;
    int k = (int)(iter % period);
    if (phase) k ^= 1;
    const int *sig = dim == 1 ? SIG1[k] : dim == 2 ? SIG2[k] : SIG3[k];
    int pp[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) pp[a] = p[a];
    for (int t = 0; t < pp[2]; ++t)
        for (int q = 0; q < pp[1]; ++q)
            for (int r = 0; r < pp[0]; ++r) {
                int s = r + pp[0] * (q + pp[1] * t);
                int sc[3] = {r, q, t};
                for (int a = 0; a < 3; ++a)
                    dirs[3 * s + a] = (int8_t)(a < dim ? sig[a] * ((sc[a] & 1) ? -1 : 1) : 1);
            }
    return OR_OK;
}

/* start corner index of a direction: bit a set when the sweep along axis a
   starts at the high end */
int or_corner(int dim, const int8_t *d)
{
    int c = 0;
    for (int a = 0; a < dim; ++a)
        if (d[a] < 0) c |= 1 << a;
    return c;
}

/* ------------------------------------------------------------------ */
/* Restricted-overlap sweep: the reading of the parallel experiments under
 * which the paper's PGS/PSOR rows (Sec. 8, Tables 1d:1-3d:3) are reproduced,
 * as opposed to the exact coupled blocks its text prescribes (Secs. 2-4).
 * Every subdomain s widens the box of its own points by `overlap` points on
 * every side (clipped to the grid) and sweeps that box lexicographically in
 * its own direction dirs[s], in place on a private copy of uold, with the
 * relaxation factor of its start corner; values outside the box are uold.
 * Only the points that s owns are kept in unew. */
int or_ras_sweep(int dim, const int64_t n[3], const int p[3], const int8_t *dirs, const double *const *diag,
                 const double *omega8, int overlap, const double *uold, const double *f, double *unew)
{
    grid_t g;
    if (overlap < 0) return OR_EINVAL;
    int st = grid_init(&g, dim, n, p);
    if (st) return st;
    double *w = (double *)malloc(sizeof(double) * g.N);
    if (!w) { grid_free(&g); return OR_ENOMEM; }
    memcpy(w, uold, sizeof(double) * g.N);
    for (int t = 0; t < g.p[2]; ++t)
        for (int q = 0; q < g.p[1]; ++q)
            for (int r = 0; r < g.p[0]; ++r) {
                const int s = r + g.p[0] * (q + g.p[1] * t);
                const int sc[3] = {r, q, t};
                const int8_t *d = dirs + 3 * s;
                const double om = omega8[or_corner(dim, d)];
                int64_t elo[3], ehi[3];
                for (int a = 0; a < 3; ++a) {
                    int64_t lo = g.lo[a][sc[a]], hi = g.hi[a][sc[a]];
                    if (a < dim) { lo -= overlap; hi += overlap; }
                    elo[a] = lo < 0 ? 0 : lo;
                    ehi[a] = hi > g.n[a] - 1 ? g.n[a] - 1 : hi;
                }
                /* the widened box starts from uold (w holds uold outside every box swept so far) */
                for (int64_t kk = elo[2]; kk <= ehi[2]; ++kk)
                    for (int64_t jj = elo[1]; jj <= ehi[1]; ++jj)
                        for (int64_t ii = elo[0]; ii <= ehi[0]; ++ii) {
                            int64_t c[3] = {ii, jj, kk};
                            int64_t P = index_of(&g, c);
                            w[P] = uold[P];
                        }
                /* lexicographic sweep of the box in direction d; neighbours outside the box read uold */
                for (int64_t k0 = 0; k0 <= ehi[2] - elo[2]; ++k0)
                    for (int64_t j0 = 0; j0 <= ehi[1] - elo[1]; ++j0)
                        for (int64_t i0 = 0; i0 <= ehi[0] - elo[0]; ++i0) {
                            int64_t loc[3] = {i0, j0, k0}, c[3];
                            for (int a = 0; a < 3; ++a)
                                c[a] = (a < dim && d[a] < 0) ? ehi[a] - loc[a] : elo[a] + loc[a];
                            int64_t P = index_of(&g, c);
                            double acc = f[P];
                            for (int a = 0; a < dim; ++a)
                                for (int sd = -1; sd <= 1; sd += 2) {
                                    int64_t qn[3] = {c[0], c[1], c[2]};
                                    qn[a] += sd;
                                    if (qn[a] < 0 || qn[a] >= g.n[a]) continue;
                                    int inside = 1;
                                    for (int b = 0; b < dim; ++b)
                                        if (qn[b] < elo[b] || qn[b] > ehi[b]) inside = 0;
                                    int64_t Q = index_of(&g, qn);
                                    acc += diag[dk(a, sd)][P] * (inside ? w[Q] : uold[Q]);
                                }
                            double scl = om / diag[0][P];
                            w[P] = (1.0 - om) * w[P] + scl * acc;
                        }
                /* keep the points s owns */
                for (int64_t kk = g.lo[2][sc[2]]; kk <= g.hi[2][sc[2]]; ++kk)
                    for (int64_t jj = g.lo[1][sc[1]]; jj <= g.hi[1][sc[1]]; ++jj)
                        for (int64_t ii = g.lo[0][sc[0]]; ii <= g.hi[0][sc[0]]; ++ii) {
                            int64_t c[3] = {ii, jj, kk};
                            int64_t P = index_of(&g, c);
                            unew[P] = w[P];
                        }
                /* restore uold in the box for the next subdomain's neighbours-outside reads */
                for (int64_t kk = elo[2]; kk <= ehi[2]; ++kk)
                    for (int64_t jj = elo[1]; jj <= ehi[1]; ++jj)
                        for (int64_t ii = elo[0]; ii <= ehi[0]; ++ii) {
                            int64_t c[3] = {ii, jj, kk};
                            int64_t P = index_of(&g, c);
                            w[P] = uold[P];
                        }
            }
    free(w);
    grid_free(&g);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Plain operations used by the drivers.                               */

int or_spmv(int dim, const int64_t n[3], const double *const *diag, const double *x, double *y)
{
    grid_t g;
    int p1[3] = {1, 1, 1};
    int st = grid_init(&g, dim, n, p1);
    if (st) return st;
    for (int64_t P = 0; P < g.N; ++P) {
        int64_t c[3];
        coords_of(&g, P, c);
        double acc = diag[0][P] * x[P];
        for (int a = 0; a < dim; ++a)
            for (int s = -1; s <= 1; s += 2) {
                int64_t q[3] = {c[0], c[1], c[2]};
                q[a] += s;
                if (q[a] < 0 || q[a] >= g.n[a]) continue;
                acc -= diag[dk(a, s)][P] * x[index_of(&g, q)];
            }
        y[P] = acc;
    }
    grid_free(&g);
    return OR_OK;
}

/* Diagonals of the variable-coefficient operator -div(alpha grad u) + beta u
 * on a unit-spaced grid (eq. d2d with delta = 1; 1D eq. d1d; Sec. 7 general
 * molecule).  alpha[a] holds the axis-a coefficient on all (n+2)^dim nodes,
 * boundary ring included, node (i,j,k) at i + (n0+2)*(j + (n1+2)*k) with
 * interior point x at node x+1.  Face values are harmonic means of the two
 * node values; a^P is the sum of the face couplings plus beta. */
int or_assemble(int dim, const int64_t n[3], const double *const *alpha, double beta,
                double *const *diag)
{
    grid_t g;
    int p1[3] = {1, 1, 1};
    int st = grid_init(&g, dim, n, p1);
    if (st) return st;
    int64_t m[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) m[a] = g.n[a] + 2;
    for (int64_t P = 0; P < g.N; ++P) {
        int64_t c[3];
        coords_of(&g, P, c);
        int64_t nd[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a) nd[a] = c[a] + 1;
        int64_t node = nd[0] + m[0] * (nd[1] + m[1] * nd[2]);
        double sum = 0.0;
        for (int a = 0; a < dim; ++a)
            for (int s = -1; s <= 1; s += 2) {
                int64_t q[3] = {nd[0], nd[1], nd[2]};
                q[a] += s;
                int64_t nb = q[0] + m[0] * (q[1] + m[1] * q[2]);
                double ap = alpha[a][node], aq = alpha[a][nb];
                double face = 2.0 * ap * aq / (ap + aq);
                diag[dk(a, s)][P] = face;
                sum += face;
            }
        diag[0][P] = sum + beta;
    }
    grid_free(&g);
    return OR_OK;
}

/* Lexicographic directional SOR, in place (eqs. 1d:sorl/sorr, sor2d_*):
 * visit the points with every axis a reversed where d[a] = -1; each update
 * uses the freshest value of every neighbour. */
int or_sor_lex(int dim, const int64_t n[3], const double *const *diag, double omega,
               const int8_t *d, const double *f, double *u)
{
    grid_t g;
    int p1[3] = {1, 1, 1};
    int st = grid_init(&g, dim, n, p1);
    if (st) return st;
    for (int64_t kk = 0; kk < g.n[2]; ++kk)
        for (int64_t jj = 0; jj < g.n[1]; ++jj)
            for (int64_t ii = 0; ii < g.n[0]; ++ii) {
                int64_t c[3] = {ii, jj, kk};
                for (int a = 0; a < 3; ++a)
                    if (a < dim && d[a] < 0) c[a] = g.n[a] - 1 - c[a];
                int64_t P = index_of(&g, c);
                double acc = f[P];
                for (int a = 0; a < dim; ++a)
                    for (int s = -1; s <= 1; s += 2) {
                        int64_t q[3] = {c[0], c[1], c[2]};
                        q[a] += s;
                        if (q[a] < 0 || q[a] >= g.n[a]) continue;
                        acc += diag[dk(a, s)][P] * u[index_of(&g, q)];
                    }
                double sc = omega / diag[0][P];
                u[P] = (1.0 - omega) * u[P] + sc * acc;
            }
    grid_free(&g);
    return OR_OK;
}

/* ------------------------------------------------------------------ */
/* Coupled blocks and the global block order.                           */

typedef struct {
    int64_t nblk;
    int64_t *off;   /* nblk+1 offsets into cells */
    int64_t *cells; /* N point indices */
} order_t;

static void order_free(order_t *o)
{
    free(o->off); free(o->cells);
    o->off = o->cells = NULL;
}

/* Block containing P: P shifted against its direction across every subset
 * of the axes whose start face P lies on and whose neighbour exists. */
static int block_of(const grid_t *g, const int8_t *dirs, int64_t P, int64_t *out)
{
    int64_t c[3];
    coords_of(g, P, c);
    int s = sub_of(g, c);
    const int8_t *d = dirs + 3 * s;
    int sc[3] = {g->own[0][c[0]], g->own[1][c[1]], g->own[2][c[2]]};
    int axes[3], na = 0;
    for (int a = 0; a < g->dim; ++a) {
        int64_t start = d[a] > 0 ? g->lo[a][sc[a]] : g->hi[a][sc[a]];
        int64_t nb = c[a] - d[a];
        if (c[a] == start && nb >= 0 && nb < g->n[a]) axes[na++] = a;
    }
    int m = 1 << na;
    for (int mask = 0; mask < m; ++mask) {
        int64_t q[3] = {c[0], c[1], c[2]};
        for (int b = 0; b < na; ++b)
            if (mask & (1 << b)) q[axes[b]] -= d[axes[b]];
        out[mask] = index_of(g, q);
    }
    return m;
}

/* Global order: subdomains by id; inside each, points in the subdomain's own
 * sweep order; a block is emitted at the first of its points reached.  Every
 * block depends only on blocks emitted before it, so a forward substitution
 * over this order computes the decomposed sweep, and a backward substitution
 * over the reversed order solves the transposed system (the permutation of
 * Sec. 5, Lemma 2d:4 / Corollary 2d:5, which makes the splitting matrices
 * block triangular). */
static int build_order(const grid_t *g, const int8_t *dirs, order_t *o)
{
    o->off = (int64_t *)malloc(sizeof(int64_t) * (g->N + 1));
    o->cells = (int64_t *)malloc(sizeof(int64_t) * g->N);
    char *done = (char *)calloc((size_t)g->N, 1);
    if (!o->off || !o->cells || !done) { free(done); order_free(o); return OR_ENOMEM; }
    int64_t nb = 0, nc = 0;
    o->off[0] = 0;
    for (int t = 0; t < g->p[2]; ++t)
        for (int q = 0; q < g->p[1]; ++q)
            for (int r = 0; r < g->p[0]; ++r) {
                int s = r + g->p[0] * (q + g->p[1] * t);
                const int8_t *d = dirs + 3 * s;
                int sc[3] = {r, q, t};
                int64_t len[3];
                for (int a = 0; a < 3; ++a) len[a] = g->hi[a][sc[a]] - g->lo[a][sc[a]] + 1;
                for (int64_t kk = 0; kk < len[2]; ++kk)
                    for (int64_t jj = 0; jj < len[1]; ++jj)
                        for (int64_t ii = 0; ii < len[0]; ++ii) {
                            int64_t loc[3] = {ii, jj, kk}, c[3];
                            for (int a = 0; a < 3; ++a)
                                c[a] = d[a] > 0 ? g->lo[a][sc[a]] + loc[a] : g->hi[a][sc[a]] - loc[a];
                            int64_t P = index_of(g, c);
                            if (done[P]) continue;
                            int64_t blk[8];
                            int m = block_of(g, dirs, P, blk);
                            for (int i = 0; i < m; ++i) {
                                done[blk[i]] = 1;
                                o->cells[nc++] = blk[i];
                            }
                            o->off[++nb] = nc;
                        }
            }
    free(done);
    o->nblk = nb;
    return nc == g->N ? OR_OK : OR_EINVAL;
}

/* Gaussian elimination with partial pivoting on an m x m system, m <= 8. */
static int gepp(int m, double A[8][8], double *b)
{
    for (int k = 0; k < m; ++k) {
        int piv = k;
        for (int i = k + 1; i < m; ++i)
            if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
        if (A[piv][k] == 0.0) return OR_ESINGULAR;
        if (piv != k) {
            for (int j = 0; j < m; ++j) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int i = k + 1; i < m; ++i) {
            double l = A[i][k] / A[k][k];
            if (l == 0.0) continue;
            for (int j = k; j < m; ++j) A[i][j] -= l * A[k][j];
            b[i] -= l * b[k];
        }
    }
    for (int i = m - 1; i >= 0; --i) {
        double acc = b[i];
        for (int j = i + 1; j < m; ++j) acc -= A[i][j] * b[j];
        b[i] = acc / A[i][i];
    }
    return OR_OK;
}

static inline int find_in(const int64_t *blk, int m, int64_t P)
{
    for (int i = 0; i < m; ++i)
        if (blk[i] == P) return i;
    return -1;
}

/* One decomposed sweep (the paper's parallel SOR update, Secs. 2-4).
 * For every point P with direction d_P (its subdomain's), relaxation w_P and
 * pivot D_P:
 *   x_P = (1-w_P) uold_P + (w_P/D_P) (f_P + sum_{upstream X} a^X_P x_X
 *                                         + sum_{downstream X} a^X_P uold_X)
 * with D_P = piv[P] if piv is given, else a^P_P; w_P = omega[corner(d_P)] if
 * omega is given, else 1; uold = 0 if NULL.  Coupled points are solved
 * jointly.  With piv given, omega NULL and uold NULL this solves
 * (Piv - N) x = f, N being the upstream couplings under dirs. */
int or_dsweep(int dim, const int64_t n[3], const int p[3], const int8_t *dirs,
              const double *const *diag, const double *piv, const double *omega,
              const double *uold, const double *f, double *xnew)
{
    grid_t g;
    int st = grid_init(&g, dim, n, p);
    if (st) return st;
    order_t o;
    st = build_order(&g, dirs, &o);
    if (st) { grid_free(&g); return st; }
    for (int64_t b = 0; b < o.nblk && st == OR_OK; ++b) {
        const int64_t *blk = o.cells + o.off[b];
        int m = (int)(o.off[b + 1] - o.off[b]);
        double A[8][8], rhs[8];
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) A[i][j] = (i == j) ? 1.0 : 0.0;
            int64_t P = blk[i], c[3];
            coords_of(&g, P, c);
            const int8_t *d = dirs + 3 * sub_of(&g, c);
            double w = omega ? omega[or_corner(dim, d)] : 1.0;
            double D = piv ? piv[P] : diag[0][P];
            double sc = w / D;
            double acc = f[P];
            for (int a = 0; a < dim; ++a)
                for (int s = -1; s <= 1; s += 2) {
                    int64_t q[3] = {c[0], c[1], c[2]};
                    q[a] += s;
                    if (q[a] < 0 || q[a] >= g.n[a]) continue;
                    int64_t Q = index_of(&g, q);
                    double coef = diag[dk(a, s)][P];
                    if (s == -d[a]) {
                        int j = find_in(blk, m, Q);
                        if (j >= 0) A[i][j] -= sc * coef;
                        else acc += coef * xnew[Q];
                    } else if (uold) {
                        acc += coef * uold[Q];
                    }
                }
            rhs[i] = uold ? (1.0 - w) * uold[P] + sc * acc : sc * acc;
        }
        if (m == 1) {
            xnew[blk[0]] = rhs[0];
        } else {
            st = gepp(m, A, rhs);
            for (int i = 0; i < m; ++i) xnew[blk[i]] = rhs[i];
        }
    }
    order_free(&o);
    grid_free(&g);
    return st;
}

/* Transposed solve (Piv - N)^T x = b, N the upstream couplings under dirs
 * (D = piv or a^P).  Row P: D_P x_P - sum_{Q : P upstream of Q} a_{Q->P} x_Q
 * = b_P, where a_{Q->P} is Q's coupling towards P.  Blocks are processed in
 * the reverse of the forward order, so the coupled blocks come last. */
int or_dsolve_t(int dim, const int64_t n[3], const int p[3], const int8_t *dirs,
                const double *const *diag, const double *piv, const double *b, double *x)
{
    grid_t g;
    int st = grid_init(&g, dim, n, p);
    if (st) return st;
    order_t o;
    st = build_order(&g, dirs, &o);
    if (st) { grid_free(&g); return st; }
    for (int64_t bb = o.nblk - 1; bb >= 0 && st == OR_OK; --bb) {
        const int64_t *blk = o.cells + o.off[bb];
        int m = (int)(o.off[bb + 1] - o.off[bb]);
        double A[8][8], rhs[8];
        for (int i = 0; i < m; ++i) {
            for (int j = 0; j < m; ++j) A[i][j] = (i == j) ? 1.0 : 0.0;
            int64_t P = blk[i], c[3];
            coords_of(&g, P, c);
            double D = piv ? piv[P] : diag[0][P];
            double sc = 1.0 / D;
            double acc = b[P];
            for (int a = 0; a < dim; ++a)
                for (int s = -1; s <= 1; s += 2) {
                    int64_t q[3] = {c[0], c[1], c[2]};
                    q[a] += s;
                    if (q[a] < 0 || q[a] >= g.n[a]) continue;
                    const int8_t *dq = dirs + 3 * sub_of(&g, q);
                    /* P = Q - s e_a is upstream of Q iff -s == -dq[a] */
                    if (s != dq[a]) continue;
                    int64_t Q = index_of(&g, q);
                    double coef = diag[dk(a, -s)][Q];
                    int j = find_in(blk, m, Q);
                    if (j >= 0) A[i][j] -= sc * coef;
                    else acc += coef * x[Q];
                }
            rhs[i] = sc * acc;
        }
        if (m == 1) {
            x[blk[0]] = rhs[0];
        } else {
            st = gepp(m, A, rhs);
            for (int i = 0; i < m; ++i) x[blk[i]] = rhs[i];
        }
    }
    order_free(&o);
    grid_free(&g);
    return st;
}

/* ILU(0) pivots of the decomposed factorisation (Sec. 5 "Parallel incomplete
 * LU"; Saad Sec. 10.3 for the recurrence):
 *   D~_P = a^P_P - sum_{Q upstream of P, same subdomain} a_{P->Q} a_{Q->P} / D~_Q
 * computed per subdomain in its sweep order.  Couplings across subdomain
 * faces contribute nothing: across a face where the lower factor couples,
 * the upper factor does not. */
int or_ilu_pivots(int dim, const int64_t n[3], const int p[3], const int8_t *dirs,
                  const double *const *diag, double *piv)
{
    grid_t g;
    int st = grid_init(&g, dim, n, p);
    if (st) return st;
    for (int t = 0; t < g.p[2] && st == OR_OK; ++t)
        for (int q = 0; q < g.p[1] && st == OR_OK; ++q)
            for (int r = 0; r < g.p[0] && st == OR_OK; ++r) {
                int s = r + g.p[0] * (q + g.p[1] * t);
                const int8_t *d = dirs + 3 * s;
                int sc[3] = {r, q, t};
                int64_t len[3];
                for (int a = 0; a < 3; ++a) len[a] = g.hi[a][sc[a]] - g.lo[a][sc[a]] + 1;
                for (int64_t kk = 0; kk < len[2]; ++kk)
                    for (int64_t jj = 0; jj < len[1]; ++jj)
                        for (int64_t ii = 0; ii < len[0]; ++ii) {
                            int64_t loc[3] = {ii, jj, kk}, c[3];
                            for (int a = 0; a < 3; ++a)
                                c[a] = d[a] > 0 ? g.lo[a][sc[a]] + loc[a] : g.hi[a][sc[a]] - loc[a];
                            int64_t P = index_of(&g, c);
                            double acc = diag[0][P];
                            for (int a = 0; a < dim; ++a) {
                                int su = -d[a]; /* side of the upstream neighbour */
                                int64_t qq[3] = {c[0], c[1], c[2]};
                                qq[a] += su;
                                if (qq[a] < 0 || qq[a] >= g.n[a]) continue;
                                if (sub_of(&g, qq) != s) continue;
                                int64_t Q = index_of(&g, qq);
                                acc -= diag[dk(a, su)][P] * diag[dk(a, -su)][Q] / piv[Q];
                            }
                            if (!(acc > 0.0)) { st = OR_EPIVOT; }
                            piv[P] = acc;
                        }
            }
    grid_free(&g);
    return st;
}
