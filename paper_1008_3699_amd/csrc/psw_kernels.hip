// psw_kernels.hip -- HIP kernels of libpsweep.so for gfx950.
//
// Decomposed sweeps (Tavakoli, Secs. 2-5).  One workgroup owns one subdomain
// ("tile").  Inside a tile the sweep advances one hyperplane level
// t = l0 + l1 + l2 at a time (the frontal strategy of Sec. 3, fig. swp2d),
// in tile-local coordinates l in which the tile's sweep runs towards +l.
// Threads own cross-section positions (l1, l2); the new value of a point is
// published in LDS where the points of the next level read it.
//
// Start-coupled passes (the paper's sweep, forward and backward
// preconditioner half-sweeps) solve the coupled blocks at the tile's start
// faces inside the tile: the partner points across a start face are
// recomputed redundantly, 2x2 on faces (eq. 1d:sorc, eq. 2d:sor2b2), 4x4 at
// 2D cross points and along 3D edges (eq. 2d:sor4b4), 8x8 at 3D corners
// (Sec. 4), so a tile needs only the old iterate and a 2-deep halo.
//
// End-coupled passes (the transpose of a start-coupled operator, used by the
// symmetric form of the preconditioner) couple at the tiles' END faces.
// They run an uncoupled interior pass first and then re-solve the coupled
// points in order of block size: faces, then edges (3D), then corners; each
// group reads only results of the earlier groups.
#include "psw_internal.h"
#include "psw_fast2d.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace psw {

// ------------------------------------------------------------------ loads
template <typename T, typename S> __device__ __forceinline__ T ldv(const S *p, int64_t i);
template <> __device__ __forceinline__ double ldv<double, double>(const double *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ldv<float, float>(const float *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ldv<float, double>(const double *p, int64_t i) { return (float)p[i]; }
template <> __device__ __forceinline__ double ldv<double, float>(const float *p, int64_t i) { return (double)p[i]; }
template <> __device__ __forceinline__ float ldv<float, uint16_t>(const uint16_t *p, int64_t i) { return bf16_to_f32(p[i]); }
// conversion of a loaded input value to the arithmetic type
template <typename T> __device__ __forceinline__ T cvt_in(double v) { return (T)v; }
template <typename T> __device__ __forceinline__ T cvt_in(float v) { return (T)v; }

// diagonal index of the coupling of a point towards its neighbour on axis a,
// side s (-1: W/S/B, +1: E/N/F)
__device__ __forceinline__ int dk(int a, int s) { return s < 0 ? 1 + 2 * a : 2 + 2 * a; }

__device__ __forceinline__ int64_t lin(const int n[3], const int g[3]) {
    return (int64_t)g[0] + (int64_t)n[0] * ((int64_t)g[1] + (int64_t)n[1] * (int64_t)g[2]);
}

struct TileFrame {
    int d[3];    // sweep direction of this tile in this pass
    int len[3];  // extent
    int base[3]; // global coordinate of local l = 0
    int lo[3];
    bool start_cpl[3]; // neighbour exists across the start side
    bool end_cpl[3];   // neighbour exists across the end side
};

template <int DIM>
__device__ __forceinline__ TileFrame make_frame(const PassGeom &g, const TileDesc &td) {
    TileFrame f;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        f.d[a] = (a < DIM) ? g.sig[a] * (td.par[a] ? -1 : 1) : 1;
        f.len[a] = td.len[a];
        f.lo[a] = td.lo[a];
        f.base[a] = f.d[a] > 0 ? td.lo[a] : td.lo[a] + td.len[a] - 1;
        bool low = td.lo[a] > 0, high = td.lo[a] + td.len[a] < g.n[a];
        f.start_cpl[a] = (a < DIM) && (f.d[a] > 0 ? low : high);
        f.end_cpl[a] = (a < DIM) && (f.d[a] > 0 ? high : low);
    }
    return f;
}

// small dense solve without pivoting, NB x NB, rows/cols outside the block
// are identity and decoupled
template <typename T, int NB>
__device__ __forceinline__ void ge_solve(T (&M)[NB][NB], T (&R)[NB]) {
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        T inv = T(1) / M[k][k];
#pragma unroll
        for (int i = k + 1; i < NB; ++i) {
            T l = M[i][k] * inv;
#pragma unroll
            for (int j = k + 1; j < NB; ++j) M[i][j] -= l * M[k][j];
            R[i] -= l * R[k];
        }
    }
#pragma unroll
    for (int i = NB - 1; i >= 0; --i) {
        T acc = R[i];
#pragma unroll
        for (int j = i + 1; j < NB; ++j) acc -= M[i][j] * R[j];
        R[i] = acc / M[i][i];
    }
}

constexpr int kWave = 64;

// Compiler-only ordering point between the levels of a loop run by one wave:
// the wave's own LDS accesses take effect in issue order, so no wait is needed.
__device__ __forceinline__ void wave_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Workgroup copy of n elements from global memory into LDS.  Each thread issues U
// loads before its first LDS store: a loop that stores every element as soon as
// it arrives waits a full memory latency per element.
template <int U, typename T>
__device__ __forceinline__ void copy_to_lds(T *__restrict__ dst, const T *__restrict__ src, int n) {
    const int nth = blockDim.x;
    for (int i0 = threadIdx.x; i0 < n; i0 += U * nth) {
        T v[U];
        // unconditional loads (an index past the end repeats the last element): a guarded load
        // becomes a branch, and the branches wait for their loads one by one
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = src[min(i0 + u * nth, n - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * nth;
            if (i < n) dst[i] = v[u];
        }
    }
}

// Workgroup barrier that orders LDS only: the waves wait for their own LDS
// accesses, not for global stores in flight.  For level loops whose global
// writes no thread of the workgroup reads back.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// LDS slot rings: one double-buffered slot per (block type B, position).
// B is the set of start-face axes a point was shifted across (0 = own point).
template <typename T> struct Rings {
    T *own, *xp, *yp, *zp, *xyp, *xzp, *yzp;
    int cmax, l1max, l2max;
    __device__ __forceinline__ T *slot(int B, int buf, int l1, int l2, int L1) const {
        switch (B) {
        case 0: return own + buf * cmax + l1 + L1 * l2;
        case 1: return xp + buf * cmax + l1 + L1 * l2;
        case 2: return yp + buf * l2max + l2;
        case 4: return zp + buf * l1max + l1;
        case 3: return xyp + buf * l2max + l2;
        case 5: return xzp + buf * l1max + l1;
        default: return yzp + buf;
        }
    }
};

template <typename T>
__device__ __forceinline__ Rings<T> make_rings(void *smem, const PassGeom &g) {
    Rings<T> r;
    T *p = reinterpret_cast<T *>(smem);
    r.cmax = g.cmax; r.l1max = g.l1max; r.l2max = g.l2max;
    r.own = p; p += 2 * g.cmax;
    r.xp = p; p += 2 * g.cmax;
    r.yp = p; p += 2 * g.l2max;
    r.zp = p; p += 2 * g.l1max;
    r.xyp = p; p += 2 * g.l2max;
    r.xzp = p; p += 2 * g.l1max;
    r.yzp = p;
    return r;
}

__host__ __device__ size_t rings_bytes(const PassGeom &g, size_t elem) {
    return elem * (size_t)(4 * g.cmax + 4 * g.l2max + 4 * g.l1max + 2);
}

// ------------------------------------------------------------------ start-coupled sweep
// STAT: stationary SOR (D = a^P, per-corner omega, old iterate uold).
// else: preconditioner half-sweep (D = piv, omega = 1, no old iterate,
//       rhs = in .* (scale_by_piv ? piv : 1), out = cscale * x).
template <typename S, typename TIN, typename TOUT> struct StartArgs {
    PassGeom g;
    const S *diag[7];
    const S *piv;
    double omega[8];
    const double *uold;
    const TIN *in;
    int scale_by_piv;
    TOUT *out;
    double cscale;
    int faces_only; // solve only the coupled blocks at the start faces (they involve no interior point)
    // coupled start faces with gathered records: 0 gather everything; 1 write the records'
    // coefficient part (pivot in place of the right-hand side) to img and stop; 2 take the
    // coefficient part from img and gather the right-hand sides only
    int img_mode;
    void *img;
    int64_t img_stride; // elements per tile
};

template <int DIM, typename T, typename S, typename TIN, typename TOUT, bool STAT>
__device__ __forceinline__ void sweep_start_body(const StartArgs<S, TIN, TOUT> &A, unsigned char *smem) {
    const PassGeom &g = A.g;
    const TileDesc td = g.tiles[blockIdx.x];
    const TileFrame F = make_frame<DIM>(g, td);
    Rings<T> rg = make_rings<T>(smem, g);
    const int L1 = F.len[1], L2 = F.len[2];
    const int C = L1 * L2;
    int nlev = F.len[0] + F.len[1] + F.len[2] - 2;
    if (!STAT && A.faces_only) {
        // the last level holding a point of a coupled start face (l_a = 0): len_b + len_c - 2
        int m = -1;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            if (F.start_cpl[a]) m = max(m, F.len[0] + F.len[1] + F.len[2] - F.len[a] - 2);
        nlev = m + 1;
    }
    constexpr int NB = 1 << DIM;

    for (int t = 0; t < nlev; ++t) {
        const int cur = t & 1, prv = cur ^ 1;
        for (int c = threadIdx.x; c < C; c += blockDim.x) {
            const int l1 = c % L1, l2 = c / L1, l0 = t - l1 - l2;
            if (l0 < 0 || l0 >= F.len[0]) continue;
            const int l[3] = {l0, l1, l2};
            int gp[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gp[a] = F.base[a] + F.d[a] * l[a];
            int Am = 0;
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                if (l[a] == 0 && F.start_cpl[a]) Am |= 1 << a;

            if (Am == 0) {
                if (!STAT && A.faces_only) continue;
                // interior point: single update
                const int64_t P = lin(g.n, gp);
                int corner = 0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) corner |= (F.d[a] < 0) << a;
                T w = STAT ? (T)A.omega[corner] : T(1);
                T D = STAT ? ldv<T>(A.diag[0], P) : ldv<T>(A.piv, P);
                T sc = w / D;
                T acc = ldv<T>(A.in, P);
                if (!STAT && A.scale_by_piv) acc *= D;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const int su = -F.d[a];
                    if (l[a] > 0) {
                        T coef = ldv<T>(A.diag[dk(a, su)], P);
                        T v = *rg.slot(0, prv, l1 - (a == 1), l2 - (a == 2), L1);
                        acc += coef * v;
                    }
                    if (STAT) {
                        int q[3] = {gp[0], gp[1], gp[2]};
                        q[a] += F.d[a];
                        if (q[a] >= 0 && q[a] < g.n[a]) acc += ldv<T>(A.diag[dk(a, F.d[a])], P) * ldv<T>(A.uold, lin(g.n, q));
                    }
                }
                T x = STAT ? (T(1) - w) * ldv<T>(A.uold, P) + sc * acc : sc * acc;
                *rg.slot(0, cur, l1, l2, L1) = x;
                A.out[P] = (TOUT)((T)A.cscale * x);
            } else {
                // one member of the coupled block: block point B (partner across the start
                // faces in B); returns its right-hand side, its coupling to the partner across
                // the single coupled face `cross` in mx (the generic path below keeps all of them)
                auto member = [&](int B, T &mx) -> T {
                    int gq[3], dq[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const bool fl = (B >> a) & 1;
                        gq[a] = gp[a] - (fl ? F.d[a] : 0);
                        dq[a] = fl ? -F.d[a] : F.d[a];
                    }
                    const int64_t Q = lin(g.n, gq);
                    int corner = 0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) corner |= (dq[a] < 0) << a;
                    const T w = STAT ? (T)A.omega[corner] : T(1);
                    const T D = STAT ? ldv<T>(A.diag[0], Q) : ldv<T>(A.piv, Q);
                    const T sc = w / D;
                    T acc = ldv<T>(A.in, Q);
                    if (!STAT && A.scale_by_piv) acc *= D;
                    mx = T(0);
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        const int su = -dq[a];
                        int q[3] = {gq[0], gq[1], gq[2]};
                        q[a] += su;
                        if (q[a] >= 0 && q[a] < g.n[a]) {
                            const T coef = ldv<T>(A.diag[dk(a, su)], Q);
                            if ((Am >> a) & 1) {
                                mx -= sc * coef;
                            } else {
                                const T v = *rg.slot(B, prv, l1 - (a == 1), l2 - (a == 2), L1);
                                acc += coef * v;
                            }
                        }
                        if (STAT) {
                            int r[3] = {gq[0], gq[1], gq[2]};
                            r[a] += dq[a];
                            if (r[a] >= 0 && r[a] < g.n[a])
                                acc += ldv<T>(A.diag[dk(a, dq[a])], Q) * ldv<T>(A.uold, lin(g.n, r));
                        }
                    }
                    return STAT ? (T(1) - w) * ldv<T>(A.uold, Q) + sc * acc : sc * acc;
                };
                if ((Am & (Am - 1)) == 0) {
                    // one coupled face: the 2x2 block (eq. 1d:sorc / eq. 2d:sor2b2) in scalars, so
                    // that nothing of it is indexed at run time
                    T m0, mb;
                    const T r0 = member(0, m0), rb = member(Am, mb);
                    const T det = T(1) - m0 * mb;
                    const T x0 = (r0 - m0 * rb) / det;
                    const T x1 = (rb - mb * r0) / det;
                    const int64_t P = lin(g.n, gp);
                    A.out[P] = (TOUT)((T)A.cscale * x0);
                    *rg.slot(0, cur, l1, l2, L1) = x0;
                    *rg.slot(Am, cur, l1, l2, L1) = x1;
                    continue;
                }
                // coupled block: own point plus partners across the coupled start faces
                T M[NB][NB], R[NB];
#pragma unroll
                for (int i = 0; i < NB; ++i) {
                    R[i] = T(0);
#pragma unroll
                    for (int j = 0; j < NB; ++j) M[i][j] = (i == j) ? T(1) : T(0);
                }
#pragma unroll
                for (int B = 0; B < NB; ++B) {
                    if (B & ~Am) continue;
                    int gq[3], dq[3];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        bool fl = (B >> a) & 1;
                        gq[a] = gp[a] - (fl ? F.d[a] : 0);
                        dq[a] = fl ? -F.d[a] : F.d[a];
                    }
                    const int64_t Q = lin(g.n, gq);
                    int corner = 0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) corner |= (dq[a] < 0) << a;
                    T w = STAT ? (T)A.omega[corner] : T(1);
                    T D = STAT ? ldv<T>(A.diag[0], Q) : ldv<T>(A.piv, Q);
                    T sc = w / D;
                    T acc = ldv<T>(A.in, Q);
                    if (!STAT && A.scale_by_piv) acc *= D;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        const int su = -dq[a];
                        int q[3] = {gq[0], gq[1], gq[2]};
                        q[a] += su;
                        if (q[a] >= 0 && q[a] < g.n[a]) {
                            T coef = ldv<T>(A.diag[dk(a, su)], Q);
                            if ((Am >> a) & 1) {
                                M[B][B ^ (1 << a)] -= sc * coef;
                            } else {
                                T v = *rg.slot(B, prv, l1 - (a == 1), l2 - (a == 2), L1);
                                acc += coef * v;
                            }
                        }
                        if (STAT) {
                            int r[3] = {gq[0], gq[1], gq[2]};
                            r[a] += dq[a];
                            if (r[a] >= 0 && r[a] < g.n[a]) acc += ldv<T>(A.diag[dk(a, dq[a])], Q) * ldv<T>(A.uold, lin(g.n, r));
                        }
                    }
                    R[B] = STAT ? (T(1) - w) * ldv<T>(A.uold, Q) + sc * acc : sc * acc;
                }
                ge_solve<T, NB>(M, R);
                const int64_t P = lin(g.n, gp);
                A.out[P] = (TOUT)((T)A.cscale * R[0]);
#pragma unroll
                for (int B = 0; B < NB - 1; ++B) {
                    if (B & ~Am) continue;
                    *rg.slot(B, cur, l1, l2, L1) = R[B];
                }
            }
        }
        lds_barrier(); // out is written, never read back, inside the sweep
    }
}

template <int DIM, typename T, typename S, typename TIN, typename TOUT, bool STAT>
__global__ void __launch_bounds__(256) k_sweep_start(StartArgs<S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_start_body<DIM, T, S, TIN, TOUT, STAT>(A, smem);
}

// the coupled start faces only, one pencil per thread (up to 1024), so that a thread
// meets at most one face point per level
template <typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(1024) k_start_faces3(StartArgs<S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    sweep_start_body<3, T, S, TIN, TOUT, false>(A, smem);
}

// The coupled start faces of a 3D preconditioner pass with their data gathered
// into LDS first.  Everything a face block needs that does not depend on the
// sweep (the right-hand sides of its points scaled by 1/Piv, and each point's
// three couplings scaled by 1/Piv) is loaded once, with all loads in flight
// together; the level loop then reads LDS and the rings only.  A point on one
// coupled face has a record of two members and the inverse determinant of its
// 2x2 block (9 values: an odd stride keeps the lanes' record reads on distinct
// LDS banks); a point on an edge or the corner has a record of eight member
// slots (indexed by the member's face bits).  An edge block uses four of the
// slots; the inverse of its 4x4 matrix goes into the other four.  Both inverses
// depend on the coefficients only and are part of the stored image.  Level
// order, ring use and block equations are those of the generic kernel.
constexpr int kRec1 = 9;  // values per single-face record
constexpr int kRecM = 32; // values per edge / corner record
// end faces: per (tile, face) image, kRec1 values per point and 2 upstream couplings across the
// face; in LDS the records and the two solved planes
constexpr int kEndImg = kRec1 + 2;

__host__ __device__ __forceinline__ int faces3_rec_floats(int len0, int len1, int len2, int lmax) {
    return kRec1 * (len1 * len2 + len0 * len2 + len0 * len1) + kRecM * (3 * lmax + 1);
}

// Rings of this kernel: the own and x-partner rings are indexed by pencil with a
// row pitch of L1 + 1, so that the lanes of the y face (one pencil row apart)
// meet distinct banks.
__host__ __device__ __forceinline__ int faces3_ring_pencils(const PassGeom &g) { return g.cmax + g.l2max; }
__host__ __device__ __forceinline__ size_t faces3_rings_elems(const PassGeom &g) {
    return (size_t)(4 * faces3_ring_pencils(g) + 4 * g.l2max + 4 * g.l1max + 2);
}

// the inverse of the 4x4 edge block: m-th member shifted across qa if m & 1 and across qb
// if m & 2; row m holds -w(member, qa) at column m ^ 1 and -w(member, qb) at column m ^ 2
template <typename T>
__device__ __forceinline__ void edge_inverse(T *rc, int qa, int qb) {
    const int qc = 3 - qa - qb;
    T M[4][4], X[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        const T *r4 = rc + 4 * (((m & 1) << qa) | ((m >> 1) << qb));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            M[m][q] = (m == q) ? T(1) : T(0);
            X[m][q] = (m == q) ? T(1) : T(0);
        }
        M[m][m ^ 1] = -r4[1 + qa];
        M[m][m ^ 2] = -r4[1 + qb];
    }
    // Gauss-Jordan without pivoting (the blocks are diagonally dominant)
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const T ip = T(1) / M[k][k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            M[k][q] *= ip;
            X[k][q] *= ip;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i == k) continue;
            const T l = M[i][k];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                M[i][q] -= l * M[k][q];
                X[i][q] -= l * X[k][q];
            }
        }
    }
    // row m of the inverse into the slot of member m shifted across qc (unused by the block)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        T *dst = rc + 4 * ((((m & 1) << qa) | ((m >> 1) << qb)) | (1 << qc));
#pragma unroll
        for (int q = 0; q < 4; ++q) dst[q] = X[m][q];
    }
}

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(1024) k_start_faces3g(StartArgs<S, TIN, TOUT> A, int lmax) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PassGeom &g = A.g;
    const TileDesc td = g.tiles[blockIdx.x];
    const TileFrame F = make_frame<3>(g, td);
    const int len[3] = {F.len[0], F.len[1], F.len[2]};
    const int L1 = len[1];
    const int PC = faces3_ring_pencils(g), RP = L1 + 1;
    T *const rown = reinterpret_cast<T *>(smem);
    T *const rxp = rown + 2 * PC;
    T *const ryp = rxp + 2 * PC;
    T *const rzp = ryp + 2 * g.l2max;
    T *const rxyp = rzp + 2 * g.l1max;
    T *const rxzp = rxyp + 2 * g.l2max;
    T *const ryzp = rxzp + 2 * g.l1max;
    const size_t nring = faces3_rings_elems(g);
    const size_t rb = (nring * sizeof(T) + 15) / 16 * 16;
    // rings start at zero: a weight of zero (no upstream point) then meets a finite value
    for (size_t i = threadIdx.x; i < nring; i += blockDim.x) rown[i] = T(0);
    T *rec1 = reinterpret_cast<T *>(smem + rb);                      // single-face records
    const int nf[3] = {len[1] * len[2], len[0] * len[2], len[0] * len[1]};
    T *recm = rec1 + kRec1 * (nf[0] + nf[1] + nf[2]);                 // edge / corner records
    const int nth = blockDim.x;
    const bool scale = A.scale_by_piv != 0;

    // face a, index j -> local point (scalars) and its coupled-face mask; owned by the lowest
    // coupled face.  Scalars only: an array selected at run time would live in scratch memory.
    auto point = [&](int a, int j, int &l0, int &l1, int &l2, int &Am) -> bool {
        if (a == 0) {
            l0 = 0;
            l1 = j % len[1];
            l2 = j / len[1];
        } else if (a == 1) {
            l1 = 0;
            l0 = j % len[0];
            l2 = j / len[0];
        } else {
            l2 = 0;
            l0 = j % len[0];
            l1 = j / len[0];
        }
        Am = (l0 == 0 && F.start_cpl[0] ? 1 : 0) | (l1 == 0 && F.start_cpl[1] ? 2 : 0) |
             (l2 == 0 && F.start_cpl[2] ? 4 : 0);
        return F.start_cpl[a] && (Am & ((1 << a) - 1)) == 0;
    };
    auto rec_of = [&](int a, int j, int l0, int l1, int l2, int Am) -> T * {
        if ((Am & (Am - 1)) == 0) {
            const int off = a == 0 ? 0 : (a == 1 ? nf[0] : nf[0] + nf[1]);
            return rec1 + kRec1 * (off + j);
        }
        if (Am == 7) return recm + kRecM * (3 * lmax);
        const int e = Am == 3 ? 0 : (Am == 5 ? 1 : 2); // x-y edge (along z), x-z (along y), y-z (along x)
        const int pos = Am == 3 ? l2 : (Am == 5 ? l1 : l0);
        return recm + kRecM * (e * lmax + pos);
    };
    // global index of member B of the block at local point (l0, l1, l2): the point shifted
    // one step against the sweep across every start face in B
    auto member_index = [&](int l0, int l1, int l2, int B) -> int64_t {
        const int gq[3] = {F.base[0] + F.d[0] * l0 - (((B >> 0) & 1) ? F.d[0] : 0),
                           F.base[1] + F.d[1] * l1 - (((B >> 1) & 1) ? F.d[1] : 0),
                           F.base[2] + F.d[2] * l2 - (((B >> 2) & 1) ? F.d[2] : 0)};
        return lin(g.n, gq);
    };
    // member B of the block at local point (l0, l1, l2): r = rhs / Piv, w[a] = coupling along a / Piv
    auto gather = [&](int l0, int l1, int l2, int B, T *r4, bool coef_only) {
        const int l[3] = {l0, l1, l2};
        int gq[3], dq[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const bool fl = (B >> a) & 1;
            gq[a] = F.base[a] + F.d[a] * l[a] - (fl ? F.d[a] : 0);
            dq[a] = fl ? -F.d[a] : F.d[a];
        }
        const int64_t Q = lin(g.n, gq);
        const T D = ldv<T>(A.piv, Q);
        const T sc = T(1) / D;
        if (coef_only) {
            r4[0] = D;
        } else {
            T acc = ldv<T>(A.in, Q);
            if (scale) acc *= D;
            r4[0] = sc * acc;
        }
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int su = -dq[a];
            int q[3] = {gq[0], gq[1], gq[2]};
            q[a] += su;
            r4[1 + a] = (q[a] >= 0 && q[a] < g.n[a]) ? sc * ldv<T>(A.diag[dk(a, su)], Q) : T(0);
        }
    };
    // the right-hand side of a member from its input value and its pivot, left in r4[0] by the
    // coefficient image (the same operations as in gather)
    auto rhs_from = [&](T *r4, TIN v) {
        const T D = r4[0];
        const T sc = T(1) / D;
        T acc = cvt_in<T>(v);
        if (scale) acc *= D;
        r4[0] = sc * acc;
    };
    // every member of every block owned by this tile's coupled start faces
    auto members = [&](auto fn) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!F.start_cpl[a]) continue;
            for (int j = threadIdx.x; j < nf[a]; j += nth) {
                int l0, l1, l2, Am;
                if (!point(a, j, l0, l1, l2, Am)) continue;
                T *rc = rec_of(a, j, l0, l1, l2, Am);
                if ((Am & (Am - 1)) == 0) {
                    fn(l0, l1, l2, 0, rc);
                    fn(l0, l1, l2, Am, rc + 4);
                } else {
#pragma unroll
                    for (int B = 0; B < 8; ++B)
                        if (!(B & ~Am)) fn(l0, l1, l2, B, rc + 4 * B);
                }
            }
        }
    };
    // the sweep-independent parts of the records: 1/det of the 2x2 blocks, the 4x4 inverses
    auto finalize = [&]() {
        members([&](int l0, int l1, int l2, int B, T *r4) {
            int Am = (l0 == 0 && F.start_cpl[0] ? 1 : 0) | (l1 == 0 && F.start_cpl[1] ? 2 : 0) |
                     (l2 == 0 && F.start_cpl[2] ? 4 : 0);
            if (B != 0) return; // once per block
            if ((Am & (Am - 1)) == 0) {
                const int bit = Am == 1 ? 0 : (Am == 2 ? 1 : 2);
                r4[8] = T(1) / (T(1) - r4[1 + bit] * r4[4 + 1 + bit]);
            } else if (Am != 7) {
                edge_inverse<T>(r4, (Am & 1) ? 0 : 1, (Am & 4) ? 2 : 1);
            }
        });
    };

    // ---- gather
    const int nrec = faces3_rec_floats(len[0], len[1], len[2], lmax);
    T *img = A.img_mode ? reinterpret_cast<T *>(A.img) + (int64_t)blockIdx.x * A.img_stride : nullptr;
    if (A.img_mode == 2) {
        // the coefficients as stored (one contiguous read per tile), then the right-hand sides,
        // every thread's loads issued before its first record update (a load index that is not
        // needed repeats the tile's first point)
        copy_to_lds<16>(rec1, img, nrec);
        __syncthreads(); // a record's pivot is read by the thread of its point, not by its copier
        const int64_t i0 = member_index(0, 0, 0, 0);
        for (int j = threadIdx.x; j < max(nf[0], max(nf[1], nf[2])); j += nth) {
            TIN v[3][2];
            bool ok[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                int l0 = 0, l1 = 0, l2 = 0, Am = 0;
                ok[a] = j < nf[a] && point(a, j, l0, l1, l2, Am) && (Am & (Am - 1)) == 0;
                v[a][0] = A.in[ok[a] ? member_index(l0, l1, l2, 0) : i0];
                v[a][1] = A.in[ok[a] ? member_index(l0, l1, l2, 1 << a) : i0];
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (!ok[a]) continue;
                int l0, l1, l2, Am;
                point(a, j, l0, l1, l2, Am);
                T *rc = rec_of(a, j, l0, l1, l2, Am);
                rhs_from(rc, v[a][0]);
                rhs_from(rc + 4, v[a][1]);
            }
        }
        // edges (thread k < 3 lmax: edge k / lmax at position k % lmax) and the corner (k = 3 lmax)
        for (int k = threadIdx.x; k <= 3 * lmax; k += nth) {
            const int e = k / lmax, pos = k - e * lmax;
            const int l0 = e == 2 ? pos : 0, l1 = e == 1 ? pos : 0, l2 = e == 0 ? pos : 0;
            const int Am = (l0 == 0 && F.start_cpl[0] ? 1 : 0) | (l1 == 0 && F.start_cpl[1] ? 2 : 0) |
                           (l2 == 0 && F.start_cpl[2] ? 4 : 0);
            const int want = e == 0 ? 3 : (e == 1 ? 5 : (e == 2 ? 6 : 7));
            const bool ok = Am == want && l0 < len[0] && l1 < len[1] && l2 < len[2];
            TIN v[8];
#pragma unroll
            for (int B = 0; B < 8; ++B) v[B] = A.in[(ok && !(B & ~Am)) ? member_index(l0, l1, l2, B) : i0];
            if (!ok) continue;
            T *rc = recm + kRecM * (e == 3 ? 3 * lmax : e * lmax + pos);
#pragma unroll
            for (int B = 0; B < 8; ++B)
                if (!(B & ~Am)) rhs_from(rc + 4 * B, v[B]);
        }
    } else {
        const bool coef_only = A.img_mode == 1;
        members([&](int l0, int l1, int l2, int B, T *r4) { gather(l0, l1, l2, B, r4, coef_only); });
        __syncthreads();
        finalize();
        if (coef_only) {
            __syncthreads();
            for (int i = threadIdx.x; i < nrec; i += nth) img[i] = rec1[i];
            return;
        }
    }
    __syncthreads();

    // ---- levels: the last one holding a face point is len_b + len_c - 2
    int nlev = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
        if (F.start_cpl[a]) nlev = max(nlev, len[0] + len[1] + len[2] - len[a] - 1);
    // The points of level t on face a are (u, t - u) in the face's own (b, c) axes (b < c).
    // A barrier waits for the surviving waves only.
    const int Lm = max(len[0], max(len[1], len[2]));
    // ring slot of member B at (q1, q2), B varying over the lanes: the address by selects
    auto rslot = [&](int B, int buf, int q1, int q2) -> T * {
        T *base = B == 0 ? rown : B == 1 ? rxp : B == 2 ? ryp : B == 4 ? rzp : B == 3 ? rxyp : B == 5 ? rxzp : ryzp;
        const int off = B <= 1 ? buf * PC + q1 + RP * q2
                      : (B == 2 || B == 3) ? buf * g.l2max + q2 : (B == 4 || B == 5) ? buf * g.l1max + q1 : buf;
        return base + off;
    };
    const int scm = (F.start_cpl[0] ? 1 : 0) | (F.start_cpl[1] ? 2 : 0) | (F.start_cpl[2] ? 4 : 0);
    const int scm0 = scm & 1, scm1 = (scm >> 1) & 1, scm2 = (scm >> 2) & 1;
    // face a, position (u, v) -> local point, record index j and coupled-face mask Am
    auto locate = [&](int a, int u, int v, int &l0, int &l1, int &l2, int &j) -> int {
        const int lenb = a == 0 ? len[1] : len[0];
        l0 = a == 0 ? 0 : u;
        l1 = a == 1 ? 0 : (a == 0 ? u : v);
        l2 = a == 2 ? 0 : v;
        j = u + v * lenb;
        return (l0 == 0 ? scm0 : 0) | (l1 == 0 ? scm1 << 1 : 0) | (l2 == 0 ? scm2 << 2 : 0);
    };
    // solve the block at one point of level t, write its ring slots and its output
    auto solve_point = [&](int a, int j, int l0, int l1, int l2, int Am, int cur, int prv) {
        const T *rc = rec_of(a, j, l0, l1, l2, Am);
        // right-hand side of member B with the upstream values outside the block
        // (the three slots are read whatever the weights: a slot is always finite, and a zero
        // weight, in the block's own directions or where the upstream point does not exist,
        // adds nothing; no branch keeps the reads apart)
        auto rhs = [&](int B, const T *r4) -> T {
            const T v0 = *rslot(B, prv, l1, l2), v1 = *rslot(B, prv, max(l1 - 1, 0), l2),
                    v2 = *rslot(B, prv, l1, max(l2 - 1, 0));
            const T w0 = (Am & 1) ? T(0) : r4[1], w1 = (Am & 2) ? T(0) : r4[2], w2 = (Am & 4) ? T(0) : r4[3];
            T x = r4[0];
            x += w0 * v0;
            x += w1 * v1;
            x += w2 * v2;
            return x;
        };
        T x0;
        if ((Am & (Am - 1)) == 0) {
            const int bit = Am == 1 ? 0 : (Am == 2 ? 1 : 2);
            const T R0 = rhs(0, rc), Rb = rhs(Am, rc + 4);
            const T m0 = -rc[1 + bit], mb = -rc[4 + 1 + bit], idet = rc[8];
            x0 = (R0 - m0 * Rb) * idet;
            const T xb = (Rb - mb * R0) * idet;
            *rslot(Am, cur, l1, l2) = xb;
        } else if (Am != 7) {
            // edge: the 4x4 block over the two coupled axes qa < qb through its stored inverse
            const int qa = (Am & 1) ? 0 : 1, qb = (Am & 4) ? 2 : 1, qc = 3 - qa - qb;
            T R[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const int B = ((m & 1) << qa) | ((m >> 1) << qb);
                R[m] = rhs(B, rc + 4 * B);
            }
            T X[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                const T *iv = rc + 4 * ((((m & 1) << qa) | ((m >> 1) << qb)) | (1 << qc));
                X[m] = iv[0] * R[0] + iv[1] * R[1] + iv[2] * R[2] + iv[3] * R[3];
            }
            x0 = X[0];
#pragma unroll
            for (int m = 1; m < 4; ++m) *rslot(((m & 1) << qa) | ((m >> 1) << qb), cur, l1, l2) = X[m];
        } else {
            T M[8][8], R[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                R[i] = T(0);
#pragma unroll
                for (int k = 0; k < 8; ++k) M[i][k] = (i == k) ? T(1) : T(0);
            }
#pragma unroll
            for (int B = 0; B < 8; ++B) {
                if (B & ~Am) continue;
                const T *r4 = rc + 4 * B;
                R[B] = rhs(B, r4);
#pragma unroll
                for (int q = 0; q < 3; ++q)
                    if ((Am >> q) & 1) M[B][B ^ (1 << q)] = -r4[1 + q];
            }
            ge_solve<T, 8>(M, R);
            x0 = R[0];
#pragma unroll
            for (int B = 1; B < 7; ++B)
                if (!(B & ~Am)) *rslot(B, cur, l1, l2) = R[B];
        }
        *rslot(0, cur, l1, l2) = x0;
        const int gp[3] = {F.base[0] + F.d[0] * l0, F.base[1] + F.d[1] * l1, F.base[2] + F.d[2] * l2};
        A.out[lin(g.n, gp)] = (TOUT)((T)A.cscale * x0);
    };

    if (Lm <= kWave && nth >= 4 * kWave) {
        // Waves 0-2 take the 2x2 blocks of faces 0-2 (lane u), wave 3 the 4x4 edge blocks (lane 0:
        // the edge (0, 0, t), 1: (0, t, 0), 2: (t, 0, 0)) and the corner at level 0: every wave runs
        // one block type, so a level costs the longest of them, not their sum.  A wave is alone on
        // its SIMD, so a level costs about four cycles per instruction on the longest path: the
        // addresses of a lane's record, ring slots and output advance by fixed strides from level
        // to level and are set up once, and each member's right-hand side reads only the ring
        // slots of its upstream neighbours outside the block.
        const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
        if (w >= 4) return;
        // global index of local point (l0, l1, l2): g0 + sum l_q gs[q]
        const int64_t g0 = member_index(0, 0, 0, 0);
        const int64_t gs0 = F.d[0], gs1 = (int64_t)F.d[1] * g.n[0], gs2 = (int64_t)F.d[2] * g.n[0] * g.n[1];
        const T cs = (T)A.cscale;
        if (w < 3) {
            const int a = w;
            const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2; // in-face axes, b < c
            const int lenb = a == 0 ? len[1] : len[0], lenc = a == 2 ? len[1] : len[2];
            const int u = lane;
            // the other coupled faces through this face (their points are edge points)
            const bool cb = (scm >> b) & 1, cc = (scm >> c) & 1;
            const bool lane_ok = ((scm >> a) & 1) && u < lenb && !(u == 0 && cb);
            const int off_a = a == 0 ? 0 : (a == 1 ? nf[0] : nf[0] + nf[1]);
            // own ring: a = 0 pencil (u, v), a = 1 pencil (0, v), a = 2 pencil (v, 0)
            const int osv = a == 2 ? 1 : RP, ou = a == 0 ? u : 0;
            const int ob = a == 0 ? (u > 0 ? -1 : 0) : 0; // b-upstream: the pencil before (a = 0) or the same
            T *const pr = a == 0 ? rxp : (a == 1 ? ryp : rzp);
            const int psz = a == 0 ? PC : (a == 1 ? g.l2max : g.l1max);
            const int psv = a == 0 ? RP : 1, pu = a == 0 ? u : 0;
            const int64_t gsb = b == 0 ? gs0 : gs1, gsc = c == 1 ? gs1 : gs2;
            const int64_t gu = g0 + (int64_t)u * gsb;
            for (int t = 0; t < nlev; ++t) {
                const int cur = t & 1, prv = cur ^ 1;
                const int v = t - u;
                if (lane_ok && v >= 0 && v < lenc && !(v == 0 && cc)) {
                    const T *rc = rec1 + kRec1 * (off_a + u + v * lenb);
                    const int oi = ou + osv * v, pi = pu + psv * v;
                    const int vu = v > 0 ? 1 : 0;
                    const T *oprv = rown + prv * PC, *pprv = pr + prv * psz;
                    const T R0 = rc[0] + rc[1 + b] * oprv[oi + ob] + rc[1 + c] * oprv[oi - vu * osv];
                    const T Rb = rc[4] + rc[5 + b] * pprv[pi + ob] + rc[5 + c] * pprv[pi - vu * psv];
                    const T idet = rc[8];
                    const T x0 = (R0 + rc[1 + a] * Rb) * idet;
                    const T xb = (Rb + rc[5 + a] * R0) * idet;
                    rown[cur * PC + oi] = x0;
                    pr[cur * psz + pi] = xb;
                    A.out[gu + (int64_t)v * gsc] = (TOUT)(cs * x0);
                }
                lds_barrier(); // out is written, never read back, inside the sweep
            }
            return;
        }
        // edges: lane e runs the edge along axis c with the coupled faces qa < qb
        const int e = lane;
        const int qa = e == 2 ? 1 : 0, qb = e == 0 ? 1 : 2, c = 3 - qa - qb;
        const bool edge_ok = e < 3 && ((scm >> qa) & 1) && ((scm >> qb) & 1);
        const int lenc = c == 0 ? len[0] : (c == 1 ? len[1] : len[2]);
        // member m = point shifted across qa if m & 1 and across qb if m & 2: its ring, buffer size
        // and index stride along the edge
        const int B1 = 1 << qa, B2 = 1 << qb, B3 = B1 | B2;
        auto ring_of = [&](int B) -> T * {
            return B == 0 ? rown : B == 1 ? rxp : B == 2 ? ryp : B == 4 ? rzp : B == 3 ? rxyp : B == 5 ? rxzp : ryzp;
        };
        auto size_of = [&](int B) -> int {
            return B <= 1 ? PC : (B == 2 || B == 3) ? g.l2max : (B == 4 || B == 5) ? g.l1max : 1;
        };
        // own and x-partner rings index pencils (l1 + RP l2), the others one coordinate
        auto stride_of = [&](int B) -> int { return B <= 1 ? (c == 2 ? RP : (c == 1 ? 1 : 0)) : (c == 0 ? 0 : 1); };
        T *const m0r = ring_of(0), *const m1r = ring_of(B1), *const m2r = ring_of(B2), *const m3r = ring_of(B3);
        const int z0 = size_of(0), z1 = size_of(B1), z2 = size_of(B2), z3 = size_of(B3);
        const int s0 = stride_of(0), s1 = stride_of(B1), s2 = stride_of(B2), s3 = stride_of(B3);
        const int64_t gsE = c == 0 ? gs0 : (c == 1 ? gs1 : gs2);
        const int qc = c;
        for (int t = 0; t < nlev; ++t) {
            const int cur = t & 1, prv = cur ^ 1;
            if (t == 0) {
                // the corner, or the start of the one edge through it: the general block solve
                if (lane == 0) {
                    int l0, l1, l2, j;
                    const int Am = locate(0, 0, 0, l0, l1, l2, j);
                    if (Am & (Am - 1)) solve_point(0, j, l0, l1, l2, Am, cur, prv);
                }
            } else if (edge_ok && t < lenc) {
                const T *rc = recm + kRecM * (e * lmax + t);
                const T *r0 = rc, *r1 = rc + 4 * B1, *r2 = rc + 4 * B2, *r3 = rc + 4 * B3;
                const int up = t - 1;
                T R[4];
                R[0] = r0[0] + r0[1 + c] * m0r[prv * z0 + s0 * up];
                R[1] = r1[0] + r1[1 + c] * m1r[prv * z1 + s1 * up];
                R[2] = r2[0] + r2[1 + c] * m2r[prv * z2 + s2 * up];
                R[3] = r3[0] + r3[1 + c] * m3r[prv * z3 + s3 * up];
                T X[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const T *iv = rc + 4 * ((((m & 1) << qa) | ((m >> 1) << qb)) | (1 << qc));
                    X[m] = iv[0] * R[0] + iv[1] * R[1] + iv[2] * R[2] + iv[3] * R[3];
                }
                m0r[cur * z0 + s0 * t] = X[0];
                m1r[cur * z1 + s1 * t] = X[1];
                m2r[cur * z2 + s2 * t] = X[2];
                m3r[cur * z3 + s3 * t] = X[3];
                A.out[g0 + (int64_t)t * gsE] = (TOUT)(cs * X[0]);
            }
            lds_barrier();
        }
        return;
    }
    // Any tile: thread k takes face k / Lm and u = k % Lm at every level.  Only the waves that
    // hold such threads stay; with one wave left its LDS accesses take effect in issue order.
    const int nlt = min(nth, (3 * Lm + kWave - 1) / kWave * kWave);
    if ((int)threadIdx.x >= nlt) return;
    for (int t = 0; t < nlev; ++t) {
        const int cur = t & 1, prv = cur ^ 1;
        for (int k = threadIdx.x; k < 3 * Lm; k += nlt) {
            const int a = k / Lm, u = k - a * Lm;
            if (!((scm >> a) & 1)) continue;
            const int lenb = a == 0 ? len[1] : len[0], lenc = a == 2 ? len[1] : len[2];
            const int v = t - u;
            if (u >= lenb || v < 0 || v >= lenc) continue;
            int l0, l1, l2, j;
            const int Am = locate(a, u, v, l0, l1, l2, j);
            if (Am & ((1 << a) - 1)) continue; // owned by the lowest coupled face
            solve_point(a, j, l0, l1, l2, Am, cur, prv);
        }
        if (nlt > kWave) lds_barrier(); // out is written, never read back, inside the sweep
        else wave_order();
    }
}

size_t faces3_lds_bytes(const PassGeom &g, int fmax, size_t elem) {
    return (faces3_rings_elems(g) * elem + 15) / 16 * 16 + elem * (size_t)fmax;
}

// ------------------------------------------------------------------ end-coupled (transposed) sweep
template <typename S, typename TIN, typename TOUT> struct EndArgs {
    PassGeom g;
    const S *diag[7];
    const S *piv;
    const TIN *in;
    int scale_by_piv;
    TOUT *out;
    // end faces with gathered records: 0 gather everything; 1 write the coefficient part of the
    // records (pivot in place of the right-hand side, then each member's coupling to its
    // upstream point across the face axis) to img and stop; 2 take it from img
    int img_mode;
    void *img;
    int64_t img_stride; // elements per (tile, face)
};

// Interior phase: x_P = (b_P + sum_{R upstream of P in its tile} a_{R->P} x_R) / Piv_P,
// with no coupling across any face.  Points on coupled end faces get a
// provisional value that the face/edge/corner passes overwrite.
template <int DIM, typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(256) k_sweep_end_interior(EndArgs<S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PassGeom &g = A.g;
    const TileDesc td = g.tiles[blockIdx.x];
    const TileFrame F = make_frame<DIM>(g, td);
    Rings<T> rg = make_rings<T>(smem, g);
    const int L1 = F.len[1], L2 = F.len[2];
    const int C = L1 * L2;
    const int nlev = F.len[0] + F.len[1] + F.len[2] - 2;
    for (int t = 0; t < nlev; ++t) {
        const int cur = t & 1, prv = cur ^ 1;
        for (int c = threadIdx.x; c < C; c += blockDim.x) {
            const int l1 = c % L1, l2 = c / L1, l0 = t - l1 - l2;
            if (l0 < 0 || l0 >= F.len[0]) continue;
            const int l[3] = {l0, l1, l2};
            int gp[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gp[a] = F.base[a] + F.d[a] * l[a];
            const int64_t P = lin(g.n, gp);
            T D = ldv<T>(A.piv, P);
            T acc = ldv<T>(A.in, P);
            if (A.scale_by_piv) acc *= D;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                if (l[a] > 0) {
                    int r[3] = {gp[0], gp[1], gp[2]};
                    r[a] -= F.d[a];
                    T coef = ldv<T>(A.diag[dk(a, F.d[a])], lin(g.n, r));
                    acc += coef * *rg.slot(0, prv, l1 - (a == 1), l2 - (a == 2), L1);
                }
            }
            T x = acc / D;
            *rg.slot(0, cur, l1, l2, L1) = x;
            A.out[P] = (TOUT)x;
        }
        __syncthreads();
    }
}

// One coupled end block.  P (global gp, tile-local l) lies on the end faces
// of the axes in Am of a tile sweeping along d.  Block points Q_B = P + sum
// over a in B of d_a e_a; each has its own tile's direction (d flipped on B).
// Row of Q: Piv_Q x_Q - sum_{a in Am} a_{Q_{B^a}->Q} x_{Q_{B^a}}
//           - sum_a [R_a is a dependency] a_{R_a->Q} x_{R_a} = b_Q,
// R_a = Q - dq_a e_a (upstream inside Q's tile); values of R_a come from x.
template <int DIM, typename T, typename S, typename TIN, typename TOUT>
__device__ void end_block(const EndArgs<S, TIN, TOUT> &A, const int gp[3], const int l[3], const int d[3],
                          int Am) {
    constexpr int NB = 1 << DIM;
    const PassGeom &g = A.g;
    if ((Am & (Am - 1)) == 0) {
        // one coupled face: the 2x2 block in scalars (nothing indexed at run time)
        auto member = [&](int B, T &mx, int64_t &Qo) -> T {
            int gq[3], dq[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const bool fl = (B >> a) & 1;
                gq[a] = gp[a] + (fl ? d[a] : 0);
                dq[a] = fl ? -d[a] : d[a];
            }
            const int64_t Q = lin(g.n, gq);
            Qo = Q;
            const T D = ldv<T>(A.piv, Q);
            T acc = ldv<T>(A.in, Q);
            if (A.scale_by_piv) acc *= D;
            mx = T(0);
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                if ((Am >> a) & 1) {
                    const int s2 = ((B >> a) & 1) ? -d[a] : d[a];
                    int q[3] = {gq[0], gq[1], gq[2]};
                    q[a] += s2;
                    mx -= ldv<T>(A.diag[dk(a, -s2)], lin(g.n, q)) / D;
                }
                if (((Am >> a) & 1) || l[a] > 0) {
                    int r[3] = {gq[0], gq[1], gq[2]};
                    r[a] -= dq[a];
                    const int64_t Ri = lin(g.n, r);
                    acc += ldv<T>(A.diag[dk(a, dq[a])], Ri) * ldv<T>(A.out, Ri);
                }
            }
            return acc / D;
        };
        T m0, mb;
        int64_t Q0, Qb;
        const T r0 = member(0, m0, Q0), rb = member(Am, mb, Qb);
        const T det = T(1) - m0 * mb;
        A.out[Q0] = (TOUT)((r0 - m0 * rb) / det);
        A.out[Qb] = (TOUT)((rb - mb * r0) / det);
        return;
    }
    T M[NB][NB], R[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
        R[i] = T(0);
#pragma unroll
        for (int j = 0; j < NB; ++j) M[i][j] = (i == j) ? T(1) : T(0);
    }
    int64_t idx[NB];
#pragma unroll
    for (int B = 0; B < NB; ++B) {
        idx[B] = 0;
        if (B & ~Am) continue;
        int gq[3], dq[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            bool fl = (B >> a) & 1;
            gq[a] = gp[a] + (fl ? d[a] : 0);
            dq[a] = fl ? -d[a] : d[a];
        }
        const int64_t Q = lin(g.n, gq);
        idx[B] = Q;
        T D = ldv<T>(A.piv, Q);
        T acc = ldv<T>(A.in, Q);
        if (A.scale_by_piv) acc *= D;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            if ((Am >> a) & 1) {
                // block mate across the face: Q_{B^a} = Q + s e_a
                int s = ((B >> a) & 1) ? -d[a] : d[a];
                int q[3] = {gq[0], gq[1], gq[2]};
                q[a] += s;
                T coef = ldv<T>(A.diag[dk(a, -s)], lin(g.n, q));
                M[B][B ^ (1 << a)] -= coef / D;
            }
            if (((Am >> a) & 1) || l[a] > 0) {
                int r[3] = {gq[0], gq[1], gq[2]};
                r[a] -= dq[a];
                const int64_t Ri = lin(g.n, r);
                T coef = ldv<T>(A.diag[dk(a, dq[a])], Ri);
                acc += coef * ldv<T>(A.out, Ri);
            }
        }
        R[B] = acc / D;
    }
    ge_solve<T, NB>(M, R);
#pragma unroll
    for (int B = 0; B < NB; ++B)
        if (!(B & ~Am)) A.out[idx[B]] = (TOUT)R[B];
}

// Faces.  The face between tiles r and r+1 on axis a is coupled in this pass
// when tile r sweeps towards it (d_a = +1); tile r owns it.  Positions on the
// face that also lie on another coupled end face (edges) are left to the
// edge / corner passes.  2D: one thread walks the chain; 3D: one workgroup
// advances a wavefront over the face.
template <int DIM, typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(256) k_end_faces(EndArgs<S, TIN, TOUT> A) {
    const PassGeom &g = A.g;
    const int tile = blockIdx.x / DIM, a = blockIdx.x % DIM;
    const TileDesc td = g.tiles[tile];
    const TileFrame F = make_frame<DIM>(g, td);
    if (!(F.d[a] > 0 && F.end_cpl[a])) return;
    // the two other axes (b, c); c unused in 2D
    const int b = (a + 1) % DIM, c = DIM == 3 ? (a + 2) % DIM : 2;
    const int Lb = F.len[b], Lc = (DIM == 3) ? F.len[c] : 1;
    const int nb = (F.end_cpl[b] ? Lb - 1 : Lb), nc = (DIM == 3 && F.end_cpl[c]) ? Lc - 1 : Lc;
    const int nlev = nb + nc - 1;
    for (int t = 0; t < nlev; ++t) {
        for (int k = threadIdx.x; k < nc; k += blockDim.x) {
            const int lc = k, lb = t - k;
            if (lb < 0 || lb >= nb) continue;
            int l[3] = {0, 0, 0};
            l[a] = F.len[a] - 1;
            l[b] = lb;
            if (DIM == 3) l[c] = lc;
            int gp[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) gp[q] = F.base[q] + F.d[q] * l[q];
            end_block<DIM, T, S, TIN, TOUT>(A, gp, l, F.d, 1 << a);
        }
        __syncthreads();
    }
}

// Faces (3D) with the data gathered first.  Face AX of a tile sweeping towards it:
// points P = (len_AX - 1, lb, lc) with partners Q = P + d_AX e_AX; points that also
// lie on another coupled end face are left to the edge and corner kernels.  All a
// 2x2 block needs except the values of its in-face upstream neighbours is gathered
// into LDS first (the right-hand side with the upstream value across AX, the two
// in-face couplings and the cross coupling, divided by the pivot, for P and Q);
// the wavefront over (lb, lc) then touches LDS only.  Equations as in end_block.
template <int AX, typename T, typename S, typename TIN, typename TOUT>
__device__ __forceinline__ void end_face3g_body(const EndArgs<S, TIN, TOUT> &A, const TileFrame &F,
                                                unsigned char *smem) {
    constexpr int a = AX, b = (AX + 1) % 3, c = (AX + 2) % 3;
    const PassGeom &g = A.g;
    const int nb = F.end_cpl[b] ? F.len[b] - 1 : F.len[b];
    const int nc = F.end_cpl[c] ? F.len[c] - 1 : F.len[c];
    const int np = nb * nc;
    T *rec = reinterpret_cast<T *>(smem); // kRec1 values per point (8 and the inverse determinant)
    T *vP = rec + kRec1 * np, *vQ = vP + np; // solved values of the P and Q planes
    const int nth = blockDim.x;
    T *img = A.img_mode ? reinterpret_cast<T *>(A.img) + (int64_t)blockIdx.x * A.img_stride : nullptr;
    T *cup = img ? img + kRec1 * np : nullptr; // coupling to the upstream point across AX, 2 per point
    if (A.img_mode == 2) copy_to_lds<8>(rec, img, kRec1 * np);
    // the records of point j: mode 0 gathers them into LDS, mode 1 writes their coefficient part to
    // the image, mode 2 completes the right-hand sides of the records copied from it
    T *const rdst = A.img_mode == 1 ? img : rec;
    if (A.img_mode == 2) {
        __syncthreads();
        // the right-hand sides: every member's two loads in flight before the first update
        const int64_t sa = a == 0 ? (int64_t)F.d[0] : (a == 1 ? (int64_t)F.d[1] * g.n[0] : (int64_t)F.d[2] * g.n[0] * g.n[1]);
        for (int k = threadIdx.x; k < np; k += nth) {
            // consecutive threads take consecutive x where x is an in-face axis (coalesced loads);
            // record j = lb + lc nb
            int lb, lc;
            if (a == 1) {
                lc = k % nc;
                lb = k / nc;
            } else {
                lb = k % nb;
                lc = k / nb;
            }
            const int j = lb + lc * nb;
            int l[3];
            l[a] = F.len[a] - 1;
            l[b] = lb;
            l[c] = lc;
            int gp[3];
#pragma unroll
            for (int q = 0; q < 3; ++q) gp[q] = F.base[q] + F.d[q] * l[q];
            // P, its partner Q = P + d_a e_a, and the upstream points across a of each
            const int64_t P = lin(g.n, gp);
            const TIN iP = A.in[P], iQ = A.in[P + sa];
            const TOUT uP = A.out[P - sa], uQ = A.out[P + 2 * sa];
            T *rc = rec + kRec1 * j;
            const T D0 = rc[0], D1 = rc[4];
            T a0 = cvt_in<T>(iP), a1 = cvt_in<T>(iQ);
            if (A.scale_by_piv) {
                a0 *= D0;
                a1 *= D1;
            }
            a0 += cup[2 * j] * cvt_in<T>(uP);
            a1 += cup[2 * j + 1] * cvt_in<T>(uQ);
            rc[0] = a0 / D0;
            rc[4] = a1 / D1;
        }
    }
    for (int j = threadIdx.x; j < (A.img_mode == 2 ? 0 : np); j += nth) {
        int l[3];
        l[a] = F.len[a] - 1;
        l[b] = j % nb;
        l[c] = j / nb;
        int gp[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) gp[q] = F.base[q] + F.d[q] * l[q];
        T *rc = rdst + kRec1 * j;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            int gq[3] = {gp[0], gp[1], gp[2]}, dq[3] = {F.d[0], F.d[1], F.d[2]};
            if (m) {
                gq[a] += F.d[a];
                dq[a] = -F.d[a];
            }
            const int64_t Q = lin(g.n, gq);
            int r[3] = {gq[0], gq[1], gq[2]};
            r[a] -= dq[a];
            const int64_t Ri = lin(g.n, r);
            const T D = ldv<T>(A.piv, Q);
            // the upstream point across AX (inside the member's own tile, final)
            const T cu = ldv<T>(A.diag[dk(a, dq[a])], Ri);
            T acc = T(0);
            if (A.img_mode == 0) {
                acc = ldv<T>(A.in, Q);
                if (A.scale_by_piv) acc *= D;
                acc += cu * ldv<T>(A.out, Ri);
            }
            // cross coupling to the block mate
            T mx;
            {
                const int s2 = m ? -F.d[a] : F.d[a];
                int q[3] = {gq[0], gq[1], gq[2]};
                q[a] += s2;
                mx = -ldv<T>(A.diag[dk(a, -s2)], lin(g.n, q)) / D;
            }
            T wb = T(0), wc = T(0);
            if (l[b] > 0) {
                int r[3] = {gq[0], gq[1], gq[2]};
                r[b] -= dq[b];
                wb = ldv<T>(A.diag[dk(b, dq[b])], lin(g.n, r)) / D;
            }
            if (l[c] > 0) {
                int r[3] = {gq[0], gq[1], gq[2]};
                r[c] -= dq[c];
                wc = ldv<T>(A.diag[dk(c, dq[c])], lin(g.n, r)) / D;
            }
            rc[4 * m + 0] = A.img_mode == 1 ? D : acc / D;
            rc[4 * m + 1] = wb;
            rc[4 * m + 2] = wc;
            rc[4 * m + 3] = mx;
            if (A.img_mode == 1) cup[2 * j + m] = cu;
        }
        // the inverse determinant of the 2x2 block (coefficients only: part of the image)
        if (A.img_mode != 2) rc[8] = T(1) / (T(1) - rc[3] * rc[7]);
    }
    if (A.img_mode == 1) return;
    __syncthreads();
    if (threadIdx.x >= kWave) return; // level loop in wave 0 alone, as for the start faces
    // global strides of the local axes (with the sweep direction) and the point (len_a - 1, 0, 0)
    const int64_t st[3] = {F.d[0], (int64_t)F.d[1] * g.n[0], (int64_t)F.d[2] * g.n[0] * g.n[1]};
    int e0[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) e0[q] = F.base[q] + (q == a ? F.d[q] * (F.len[a] - 1) : 0);
    const int64_t g0 = lin(g.n, e0);
    const int nlev = nb + nc - 1;
    for (int t = 0; t < nlev; ++t) {
        // the points of level t: (lb, t - lb)
        for (int lb = threadIdx.x; lb < nb; lb += kWave) {
            const int lc = t - lb;
            if (lc < 0 || lc >= nc) continue;
            const int j = lb + lc * nb;
            const T *rc = rec + kRec1 * j;
            // the in-face upstream values (a weight is zero where the neighbour is outside the face;
            // the clamped index keeps the read in range and the select drops it)
            const int jb = lb > 0 ? j - 1 : j, jc = lc > 0 ? j - nb : j;
            const T pb = vP[jb], qb = vQ[jb], pc = vP[jc], qc = vQ[jc];
            T R0 = rc[0], Rb = rc[4];
            if (lb > 0) {
                R0 += rc[1] * pb;
                Rb += rc[5] * qb;
            }
            if (lc > 0) {
                R0 += rc[2] * pc;
                Rb += rc[6] * qc;
            }
            const T m0 = rc[3], mb = rc[7], idet = rc[8];
            const T x0 = (R0 - m0 * Rb) * idet;
            const T xb = (Rb - mb * R0) * idet;
            vP[j] = x0;
            vQ[j] = xb;
            const int64_t gp = g0 + lb * st[b] + lc * st[c];
            A.out[gp] = (TOUT)x0;
            A.out[gp + st[a]] = (TOUT)xb;
        }
        wave_order();
    }
}

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(1024) k_end_faces3g(EndArgs<S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tile = blockIdx.x / 3, a = blockIdx.x % 3;
    const TileFrame F = make_frame<3>(A.g, A.g.tiles[tile]);
    // the frame's arrays are read with constant indices only (a run-time index would put the
    // frame in scratch memory)
    auto owns = [&](int q) { return F.d[q] > 0 && F.end_cpl[q]; };
    if (!(a == 0 ? owns(0) : (a == 1 ? owns(1) : owns(2)))) return;
    if (a == 0) end_face3g_body<0, T, S, TIN, TOUT>(A, F, smem);
    else if (a == 1) end_face3g_body<1, T, S, TIN, TOUT>(A, F, smem);
    else end_face3g_body<2, T, S, TIN, TOUT>(A, F, smem);
}

// Edges (3D) with the data gathered first: the edge along axis CX where the end
// faces of a and b meet.  The four block points of each edge position (P and its
// partners across a, b and both) get their right-hand sides with the upstream
// values across a and b (final after the faces), their couplings along the edge
// and their cross couplings, divided by the pivot, gathered by all threads; one
// thread then runs the chain of 4x4 blocks along the edge from LDS.
template <int CX, typename T, typename S, typename TIN, typename TOUT>
__device__ __forceinline__ void end_edge3g_body(const EndArgs<S, TIN, TOUT> &A, const TileFrame &F,
                                                unsigned char *smem) {
    constexpr int c = CX, a = (CX + 1) % 3, b = (CX + 2) % 3;
    const PassGeom &g = A.g;
    const int nc = F.end_cpl[c] ? F.len[c] - 1 : F.len[c];
    T *rec = reinterpret_cast<T *>(smem); // 16 values per position: member m = (flip a) | (flip b) << 1
    for (int j = threadIdx.x; j < nc; j += blockDim.x) {
        int l[3];
        l[a] = F.len[a] - 1;
        l[b] = F.len[b] - 1;
        l[c] = j;
        int gp[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) gp[q] = F.base[q] + F.d[q] * l[q];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int gq[3] = {gp[0], gp[1], gp[2]}, dq[3] = {F.d[0], F.d[1], F.d[2]};
            if (m & 1) {
                gq[a] += F.d[a];
                dq[a] = -F.d[a];
            }
            if (m & 2) {
                gq[b] += F.d[b];
                dq[b] = -F.d[b];
            }
            const int64_t Q = lin(g.n, gq);
            const T D = ldv<T>(A.piv, Q);
            T acc = ldv<T>(A.in, Q);
            if (A.scale_by_piv) acc *= D;
            T mcr[2];
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int q = k == 0 ? a : b;
                const bool fl = k == 0 ? (m & 1) : (m & 2);
                const int s2 = fl ? -F.d[q] : F.d[q];
                int qp[3] = {gq[0], gq[1], gq[2]};
                qp[q] += s2;
                mcr[k] = -ldv<T>(A.diag[dk(q, -s2)], lin(g.n, qp)) / D;
                int r[3] = {gq[0], gq[1], gq[2]};
                r[q] -= dq[q];
                const int64_t Ri = lin(g.n, r);
                acc += ldv<T>(A.diag[dk(q, dq[q])], Ri) * ldv<T>(A.out, Ri);
            }
            T wc = T(0);
            if (l[c] > 0) {
                int r[3] = {gq[0], gq[1], gq[2]};
                r[c] -= dq[c];
                wc = ldv<T>(A.diag[dk(c, dq[c])], lin(g.n, r)) / D;
            }
            T *rc = rec + 16 * j + 4 * m;
            rc[0] = acc / D;
            rc[1] = wc;
            rc[2] = mcr[0];
            rc[3] = mcr[1];
        }
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    T xp[4] = {T(0), T(0), T(0), T(0)};
    for (int j = 0; j < nc; ++j) {
        const T *rc = rec + 16 * j;
        T M[4][4], R[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
#pragma unroll
            for (int k = 0; k < 4; ++k) M[m][k] = (m == k) ? T(1) : T(0);
            R[m] = rc[4 * m] + rc[4 * m + 1] * xp[m];
            M[m][m ^ 1] = rc[4 * m + 2];
            M[m][m ^ 2] = rc[4 * m + 3];
        }
        ge_solve<T, 4>(M, R);
        int l[3];
        l[a] = F.len[a] - 1;
        l[b] = F.len[b] - 1;
        l[c] = j;
        int gp[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) gp[q] = F.base[q] + F.d[q] * l[q];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            int gq[3] = {gp[0], gp[1], gp[2]};
            if (m & 1) gq[a] += F.d[a];
            if (m & 2) gq[b] += F.d[b];
            A.out[lin(g.n, gq)] = (TOUT)R[m];
            xp[m] = R[m];
        }
    }
}

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(64) k_end_edges3g(EndArgs<S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int tile = blockIdx.x / 3, c = blockIdx.x % 3;
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    const TileFrame F = make_frame<3>(A.g, A.g.tiles[tile]);
    auto owns = [&](int q) { return F.d[q] > 0 && F.end_cpl[q]; };
    const bool oa = a == 0 ? owns(0) : (a == 1 ? owns(1) : owns(2));
    const bool ob = b == 0 ? owns(0) : (b == 1 ? owns(1) : owns(2));
    if (!(oa && ob)) return;
    if (c == 0) end_edge3g_body<0, T, S, TIN, TOUT>(A, F, smem);
    else if (c == 1) end_edge3g_body<1, T, S, TIN, TOUT>(A, F, smem);
    else end_edge3g_body<2, T, S, TIN, TOUT>(A, F, smem);
}

// Edges (3D): the edge along axis c where the end faces of a and b meet; owned
// by the tile that sweeps towards both.  One thread walks the edge chain.
template <typename T, typename S, typename TIN, typename TOUT>
__global__ void k_end_edges(EndArgs<S, TIN, TOUT> A) {
    const PassGeom &g = A.g;
    const int id = blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= g.ntiles * 3) return;
    const int tile = id / 3, c = id % 3;
    const int a = (c + 1) % 3, b = (c + 2) % 3;
    const TileDesc td = g.tiles[tile];
    const TileFrame F = make_frame<3>(g, td);
    if (!(F.d[a] > 0 && F.end_cpl[a] && F.d[b] > 0 && F.end_cpl[b])) return;
    const int nc = F.end_cpl[c] ? F.len[c] - 1 : F.len[c];
    for (int lc = 0; lc < nc; ++lc) {
        int l[3];
        l[a] = F.len[a] - 1;
        l[b] = F.len[b] - 1;
        l[c] = lc;
        int gp[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) gp[q] = F.base[q] + F.d[q] * l[q];
        end_block<3, T, S, TIN, TOUT>(A, gp, l, F.d, (1 << a) | (1 << b));
    }
}

// Corners: where all DIM end faces are coupled; owned by the tile sweeping
// towards +x, +y (+z).
template <int DIM, typename T, typename S, typename TIN, typename TOUT>
__global__ void k_end_corners(EndArgs<S, TIN, TOUT> A) {
    const PassGeom &g = A.g;
    const int tile = blockIdx.x * blockDim.x + threadIdx.x;
    if (tile >= g.ntiles) return;
    const TileDesc td = g.tiles[tile];
    const TileFrame F = make_frame<DIM>(g, td);
    int Am = 0;
    for (int a = 0; a < DIM; ++a) {
        if (!(F.d[a] > 0 && F.end_cpl[a])) return;
        Am |= 1 << a;
    }
    int l[3] = {0, 0, 0}, gp[3];
    for (int a = 0; a < 3; ++a) {
        l[a] = a < DIM ? F.len[a] - 1 : 0;
        gp[a] = F.base[a] + F.d[a] * l[a];
    }
    end_block<DIM, T, S, TIN, TOUT>(A, gp, l, F.d, Am);
}

// ------------------------------------------------------------------ ILU(0) pivots
struct PivArgs {
    PassGeom g;
    const double *diag[7];
    double *piv;
    int *bad;
};

template <int DIM>
__global__ void __launch_bounds__(256) k_ilu_pivots(PivArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PassGeom &g = A.g;
    const TileDesc td = g.tiles[blockIdx.x];
    const TileFrame F = make_frame<DIM>(g, td);
    Rings<double> rg = make_rings<double>(smem, g);
    const int L1 = F.len[1], L2 = F.len[2];
    const int C = L1 * L2;
    const int nlev = F.len[0] + F.len[1] + F.len[2] - 2;
    for (int t = 0; t < nlev; ++t) {
        const int cur = t & 1, prv = cur ^ 1;
        for (int c = threadIdx.x; c < C; c += blockDim.x) {
            const int l1 = c % L1, l2 = c / L1, l0 = t - l1 - l2;
            if (l0 < 0 || l0 >= F.len[0]) continue;
            const int l[3] = {l0, l1, l2};
            int gp[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) gp[a] = F.base[a] + F.d[a] * l[a];
            const int64_t P = lin(g.n, gp);
            double acc = A.diag[0][P];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                if (l[a] > 0) {
                    const int su = -F.d[a];
                    int r[3] = {gp[0], gp[1], gp[2]};
                    r[a] += su;
                    const int64_t Q = lin(g.n, r);
                    double pq = *rg.slot(0, prv, l1 - (a == 1), l2 - (a == 2), L1);
                    acc -= A.diag[dk(a, su)][P] * A.diag[dk(a, -su)][Q] / pq;
                }
            }
            if (!(acc > 0.0)) atomicOr(A.bad, 1);
            *rg.slot(0, cur, l1, l2, L1) = acc;
            A.piv[P] = acc;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ launchers
static int block_threads(const PassGeom &g) {
    int t = ((g.cmax + 63) / 64) * 64;
    return t < 64 ? 64 : (t > 256 ? 256 : t);
}

hipError_t launch_sweep_stationary(const PassGeom &g, const double *const *diag, const double *omega8,
                                   const double *uold, const double *f, double *out, hipStream_t st) {
    StartArgs<double, double, double> A{};
    A.g = g;
    for (int k = 0; k < 2 * g.dim + 1; ++k) A.diag[k] = diag[k];
    A.piv = nullptr;
    for (int k = 0; k < 8; ++k) A.omega[k] = omega8[k];
    A.uold = uold;
    A.in = f;
    A.scale_by_piv = 0;
    A.out = out;
    A.cscale = 1.0;
    size_t sm = rings_bytes(g, sizeof(double));
    dim3 grid(g.ntiles), blk(block_threads(g));
    if (g.dim == 2)
        hipLaunchKernelGGL((k_sweep_start<2, double, double, double, double, true>), grid, blk, sm, st, A);
    else
        hipLaunchKernelGGL((k_sweep_start<3, double, double, double, double, true>), grid, blk, sm, st, A);
    return hipGetLastError();
}

// ---------------------------------------------------------------- restricted-overlap sweep
// The reading of the parallel experiments under which the paper's PGS/PSOR rows (Sec. 8) are
// reproduced: every subdomain sweeps its own box widened by `overlap` points on every side (clipped
// to the grid), in its own direction and with the factor of its start corner, on a private copy of
// u_old, with u_old outside the widened box; only its own points are written.  One workgroup per
// subdomain holds the widened box and a ring of one point around it in LDS and sweeps it by
// hyperplanes (a point's upstream neighbours lie on the previous hyperplane), in place.
struct RasArgs {
    PassGeom g;
    const double *diag[7];
    double omega[8];
    int overlap;
    const double *uold, *f;
    double *out;
};

template <int DIM>
__global__ void __launch_bounds__(256) k_ras(RasArgs A) {
    extern __shared__ __align__(16) unsigned char smem[];
    double *box = reinterpret_cast<double *>(smem);
    const TileDesc td = A.g.tiles[blockIdx.x];
    int d[3], elo[3], ext[3], rext[3];
    int corner = 0;
    for (int a = 0; a < 3; ++a) {
        d[a] = A.g.sig[a] * (td.par[a] ? -1 : 1);
        if (a < DIM && d[a] < 0) corner |= 1 << a;
        const int lo = a < DIM ? max(0, td.lo[a] - A.overlap) : 0;
        const int hi = a < DIM ? min(A.g.n[a] - 1, td.lo[a] + td.len[a] - 1 + A.overlap) : 0;
        elo[a] = lo;
        ext[a] = hi - lo + 1;
        rext[a] = a < DIM ? ext[a] + 2 : 1; // with the ring
    }
    const double w = A.omega[corner];
    const int n0 = A.g.n[0], n1 = A.g.n[1];
    const int64_t nr = (int64_t)rext[0] * rext[1] * rext[2];
    // ring coordinate r = box coordinate + 1 on the used axes
    auto ridx = [&](int r0, int r1, int r2) -> int { return r0 + rext[0] * (r1 + rext[1] * r2); };
    // stage u_old on the box and its ring (zero where the ring leaves the grid)
    for (int64_t e = threadIdx.x; e < nr; e += blockDim.x) {
        const int r0 = (int)(e % rext[0]), r1 = (int)((e / rext[0]) % rext[1]), r2 = (int)(e / ((int64_t)rext[0] * rext[1]));
        const int g0 = elo[0] + r0 - 1, g1 = DIM >= 2 ? elo[1] + r1 - 1 : 0, g2 = DIM >= 3 ? elo[2] + r2 - 1 : 0;
        const bool in = g0 >= 0 && g0 < n0 && (DIM < 2 || (g1 >= 0 && g1 < n1)) && (DIM < 3 || (g2 >= 0 && g2 < A.g.n[2]));
        box[e] = in ? A.uold[(int64_t)g0 + (int64_t)n0 * (g1 + (int64_t)n1 * g2)] : 0.0;
    }
    __syncthreads();
    // hyperplanes t = l0 + l1 + l2 of local coordinates in the sweep orientation
    const int nlev = ext[0] + (DIM >= 2 ? ext[1] - 1 : 0) + (DIM >= 3 ? ext[2] - 1 : 0);
    const int npen = (DIM >= 2 ? ext[1] : 1) * (DIM >= 3 ? ext[2] : 1);
    for (int t = 0; t < nlev; ++t) {
        for (int c = threadIdx.x; c < npen; c += blockDim.x) {
            const int l1 = DIM >= 2 ? c % ext[1] : 0, l2 = DIM >= 3 ? c / ext[1] : 0;
            const int l0 = t - l1 - l2;
            if (l0 < 0 || l0 >= ext[0]) continue;
            const int l[3] = {l0, l1, l2};
            int b[3], gc[3];
            for (int a = 0; a < 3; ++a) {
                b[a] = a < DIM ? (d[a] > 0 ? l[a] : ext[a] - 1 - l[a]) : 0; // box coordinate
                gc[a] = elo[a] + b[a];
            }
            const int64_t P = (int64_t)gc[0] + (int64_t)n0 * (gc[1] + (int64_t)n1 * gc[2]);
            const int rp = ridx(b[0] + 1, DIM >= 2 ? b[1] + 1 : 0, DIM >= 3 ? b[2] + 1 : 0);
            double acc = A.f[P];
            // neighbours in the order W, E, S, N, B, F; a neighbour outside the grid reads the zero ring
            acc += A.diag[1][P] * box[rp - 1];
            acc += A.diag[2][P] * box[rp + 1];
            if (DIM >= 2) {
                acc += A.diag[3][P] * box[rp - rext[0]];
                acc += A.diag[4][P] * box[rp + rext[0]];
            }
            if (DIM >= 3) {
                acc += A.diag[5][P] * box[rp - rext[0] * rext[1]];
                acc += A.diag[6][P] * box[rp + rext[0] * rext[1]];
            }
            box[rp] = (1.0 - w) * box[rp] + (w / A.diag[0][P]) * acc;
        }
        __syncthreads();
    }
    // own points back
    const int64_t own = (int64_t)td.len[0] * (DIM >= 2 ? td.len[1] : 1) * (DIM >= 3 ? td.len[2] : 1);
    for (int64_t e = threadIdx.x; e < own; e += blockDim.x) {
        const int o0 = (int)(e % td.len[0]);
        const int o1 = DIM >= 2 ? (int)((e / td.len[0]) % td.len[1]) : 0;
        const int o2 = DIM >= 3 ? (int)(e / ((int64_t)td.len[0] * td.len[1])) : 0;
        const int g0 = td.lo[0] + o0, g1 = DIM >= 2 ? td.lo[1] + o1 : 0, g2 = DIM >= 3 ? td.lo[2] + o2 : 0;
        const int rp = ridx(g0 - elo[0] + 1, DIM >= 2 ? g1 - elo[1] + 1 : 0, DIM >= 3 ? g2 - elo[2] + 1 : 0);
        A.out[(int64_t)g0 + (int64_t)n0 * (g1 + (int64_t)n1 * g2)] = box[rp];
    }
}

// LDS bytes of the widened box with its ring for the largest subdomain (0: too large for one workgroup)
size_t ras_lds_bytes(const PassGeom &g, const int lenmax[3], int overlap, size_t lds_limit) {
    size_t e = 1;
    for (int a = 0; a < g.dim; ++a) e *= (size_t)std::min(g.n[a], lenmax[a] + 2 * overlap) + 2;
    e *= sizeof(double);
    return e <= lds_limit ? e : 0;
}

hipError_t launch_ras(const PassGeom &g, const double *const *diag, const double *omega8, int overlap, size_t lds,
                      const double *uold, const double *f, double *out, hipStream_t st) {
    RasArgs A{};
    A.g = g;
    for (int k = 0; k < 2 * g.dim + 1; ++k) A.diag[k] = diag[k];
    for (int k = 0; k < 8; ++k) A.omega[k] = omega8[k];
    A.overlap = overlap;
    A.uold = uold;
    A.f = f;
    A.out = out;
    if (g.dim == 1)
        hipLaunchKernelGGL(k_ras<1>, dim3(g.ntiles), dim3(64), lds, st, A);
    else if (g.dim == 2)
        hipLaunchKernelGGL(k_ras<2>, dim3(g.ntiles), dim3(256), lds, st, A);
    else
        hipLaunchKernelGGL(k_ras<3>, dim3(g.ntiles), dim3(256), lds, st, A);
    return hipGetLastError();
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t start_impl(const PassGeom &g, const void *const *diag, const void *piv, const void *in,
                             bool scale_by_piv, void *out, double cscale, hipStream_t st, bool faces_only = false,
                             int len0max = 0, size_t lds_limit = 0, void *img = nullptr, int img_mode = 0) {
    StartArgs<S, TIN, TOUT> A{};
    A.faces_only = faces_only ? 1 : 0;
    A.g = g;
    for (int k = 0; k < 2 * g.dim + 1; ++k) A.diag[k] = (const S *)diag[k];
    A.piv = (const S *)piv;
    for (int k = 0; k < 8; ++k) A.omega[k] = 1.0;
    A.uold = nullptr;
    A.in = (const TIN *)in;
    A.scale_by_piv = scale_by_piv ? 1 : 0;
    A.out = (TOUT *)out;
    A.cscale = cscale;
    size_t sm = rings_bytes(g, sizeof(T));
    dim3 grid(g.ntiles), blk(block_threads(g));
    if (g.dim == 2)
        hipLaunchKernelGGL((k_sweep_start<2, T, S, TIN, TOUT, false>), grid, blk, sm, st, A);
    else if (faces_only && g.cmax <= 1024) {
        const int nth = std::max(64, (g.cmax + 63) / 64 * 64);
        const int lmax = std::max(len0max, std::max(g.l1max, g.l2max));
        const int fmax = faces3_rec_floats(len0max, g.l1max, g.l2max, lmax);
        const size_t smg = faces3_lds_bytes(g, fmax, sizeof(T));
        if (len0max > 0 && smg <= lds_limit) {
            A.img_mode = img ? img_mode : 0;
            A.img = img;
            A.img_stride = fmax;
            hipLaunchKernelGGL((k_start_faces3g<T, S, TIN, TOUT>), grid, dim3(nth), smg, st, A, lmax);
        } else if (img_mode == 1) {
            return hipErrorNotSupported; // no gathered-record kernel for these tiles: no image
        } else {
            hipLaunchKernelGGL((k_start_faces3<T, S, TIN, TOUT>), grid, dim3(nth), sm, st, A);
        }
    }
    else
        hipLaunchKernelGGL((k_sweep_start<3, T, S, TIN, TOUT, false>), grid, blk, sm, st, A);
    return hipGetLastError();
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t end_impl(const PassGeom &g, const void *const *diag, const void *piv, const void *in,
                           bool scale_by_piv, void *out, hipStream_t st) {
    EndArgs<S, TIN, TOUT> A{};
    A.g = g;
    for (int k = 0; k < 2 * g.dim + 1; ++k) A.diag[k] = (const S *)diag[k];
    A.piv = (const S *)piv;
    A.in = (const TIN *)in;
    A.scale_by_piv = scale_by_piv ? 1 : 0;
    A.out = (TOUT *)out;
    size_t sm = rings_bytes(g, sizeof(T));
    dim3 grid(g.ntiles), blk(block_threads(g));
    if (g.dim == 2) {
        hipLaunchKernelGGL((k_sweep_end_interior<2, T, S, TIN, TOUT>), grid, blk, sm, st, A);
        hipLaunchKernelGGL((k_end_faces<2, T, S, TIN, TOUT>), dim3(g.ntiles * 2), dim3(64), 0, st, A);
        hipLaunchKernelGGL((k_end_corners<2, T, S, TIN, TOUT>), dim3((g.ntiles + 63) / 64), dim3(64), 0, st, A);
    } else {
        hipLaunchKernelGGL((k_sweep_end_interior<3, T, S, TIN, TOUT>), grid, blk, sm, st, A);
        hipLaunchKernelGGL((k_end_faces<3, T, S, TIN, TOUT>), dim3(g.ntiles * 3), dim3(64), 0, st, A);
        hipLaunchKernelGGL((k_end_edges<T, S, TIN, TOUT>), dim3((g.ntiles * 3 + 63) / 64), dim3(64), 0, st, A);
        hipLaunchKernelGGL((k_end_corners<3, T, S, TIN, TOUT>), dim3((g.ntiles + 63) / 64), dim3(64), 0, st, A);
    }
    return hipGetLastError();
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t end_part_impl(const PassGeom &g, const void *const *diag, const void *piv, const void *in,
                                bool scale_by_piv, void *out, int part, hipStream_t st, int len0max = 0,
                                size_t lds_limit = 0, void *img = nullptr, int img_mode = 0) {
    EndArgs<S, TIN, TOUT> A{};
    A.g = g;
    for (int k = 0; k < 2 * g.dim + 1; ++k) A.diag[k] = (const S *)diag[k];
    A.piv = (const S *)piv;
    A.in = (const TIN *)in;
    A.scale_by_piv = scale_by_piv ? 1 : 0;
    A.out = (TOUT *)out;
    if (part == 0) {
        size_t sm = rings_bytes(g, sizeof(T));
        dim3 grid(g.ntiles), blk(block_threads(g));
        if (g.dim == 2) hipLaunchKernelGGL((k_sweep_end_interior<2, T, S, TIN, TOUT>), grid, blk, sm, st, A);
        else hipLaunchKernelGGL((k_sweep_end_interior<3, T, S, TIN, TOUT>), grid, blk, sm, st, A);
    } else if (part == 1) {
        if (g.dim == 2)
            hipLaunchKernelGGL((k_end_corners<2, T, S, TIN, TOUT>), dim3((g.ntiles + 63) / 64), dim3(64), 0, st, A);
        else
            hipLaunchKernelGGL((k_end_corners<3, T, S, TIN, TOUT>), dim3((g.ntiles + 63) / 64), dim3(64), 0, st, A);
    } else {
        if (g.dim != 3) return hipErrorInvalidValue;
        // largest end face: every face has at most max(len_b len_c) points
        const int fmax = std::max(g.l1max * g.l2max, len0max * std::max(g.l1max, g.l2max));
        const bool gathered = len0max > 0 && fmax <= 1024 && kEndImg * (size_t)fmax * sizeof(T) <= lds_limit;
        if (img_mode == 1) {
            // only the coefficient image of the gathered-record kernel
            if (!gathered || !img) return hipErrorNotSupported;
            A.img_mode = 1;
            A.img = img;
            A.img_stride = kEndImg * (int64_t)fmax;
            hipLaunchKernelGGL((k_end_faces3g<T, S, TIN, TOUT>), dim3(g.ntiles * 3),
                               dim3(std::max(64, (fmax + 63) / 64 * 64)), kEndImg * (size_t)fmax * sizeof(T), st, A);
            return hipGetLastError();
        }
        if (gathered) {
            A.img_mode = img ? 2 : 0;
            A.img = img;
            A.img_stride = kEndImg * (int64_t)fmax;
            hipLaunchKernelGGL((k_end_faces3g<T, S, TIN, TOUT>), dim3(g.ntiles * 3),
                               dim3(std::max(64, (fmax + 63) / 64 * 64)), kEndImg * (size_t)fmax * sizeof(T), st, A);
        } else {
            hipLaunchKernelGGL((k_end_faces<3, T, S, TIN, TOUT>), dim3(g.ntiles * 3), dim3(64), 0, st, A);
        }
        const int lmax = std::max(len0max, std::max(g.l1max, g.l2max));
        if (len0max > 0 && 16 * (size_t)lmax * sizeof(T) <= lds_limit)
            hipLaunchKernelGGL((k_end_edges3g<T, S, TIN, TOUT>), dim3(g.ntiles * 3), dim3(64),
                               16 * (size_t)lmax * sizeof(T), st, A);
        else
            hipLaunchKernelGGL((k_end_edges<T, S, TIN, TOUT>), dim3((g.ntiles * 3 + 63) / 64), dim3(64), 0, st, A);
        hipLaunchKernelGGL((k_end_corners<3, T, S, TIN, TOUT>), dim3((g.ntiles + 63) / 64), dim3(64), 0, st, A);
    }
    return hipGetLastError();
}

static hipError_t end_part(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                           bool in_f64, bool scale_by_piv, void *out, bool out_f64, int part, hipStream_t st,
                           int len0max = 0, size_t lds_limit = 0, void *img = nullptr, int img_mode = 0) {
    if (s == Store::F64) {
        if (!in_f64 || !out_f64) return hipErrorInvalidValue;
        return end_part_impl<double, double, double, double>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
    }
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return end_part_impl<float, float, double, float>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
        if (!in_f64 && !out_f64) return end_part_impl<float, float, float, float>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
        if (in_f64 && out_f64) return end_part_impl<float, float, double, double>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
        return end_part_impl<float, float, float, double>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
    }
    if (in_f64 && !out_f64) return end_part_impl<float, uint16_t, double, float>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
    if (!in_f64 && !out_f64) return end_part_impl<float, uint16_t, float, float>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
    if (in_f64 && out_f64) return end_part_impl<float, uint16_t, double, double>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
    return end_part_impl<float, uint16_t, float, double>(g, diag, piv, in, scale_by_piv, out, part, st, len0max, lds_limit, img, img_mode);
}

hipError_t launch_end_corners(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                              bool in_f64, bool scale_by_piv, void *out, bool out_f64, hipStream_t st) {
    return end_part(g, s, diag, piv, in, in_f64, scale_by_piv, out, out_f64, 1, st);
}

hipError_t launch_end_interior(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                               bool in_f64, bool scale_by_piv, void *out, bool out_f64, hipStream_t st) {
    return end_part(g, s, diag, piv, in, in_f64, scale_by_piv, out, out_f64, 0, st);
}

hipError_t launch_half_start(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                             bool in_f64, bool scale_by_piv, void *out, bool out_f64, double cscale,
                             hipStream_t st) {
    if (s == Store::F64) {
        if (!in_f64 || !out_f64) return hipErrorInvalidValue;
        return start_impl<double, double, double, double>(g, diag, piv, in, scale_by_piv, out, cscale, st);
    }
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return start_impl<float, float, double, float>(g, diag, piv, in, scale_by_piv, out, cscale, st);
        if (!in_f64 && out_f64) return start_impl<float, float, float, double>(g, diag, piv, in, scale_by_piv, out, cscale, st);
        if (in_f64 && out_f64) return start_impl<float, float, double, double>(g, diag, piv, in, scale_by_piv, out, cscale, st);
        return start_impl<float, float, float, float>(g, diag, piv, in, scale_by_piv, out, cscale, st);
    }
    if (in_f64 && !out_f64) return start_impl<float, uint16_t, double, float>(g, diag, piv, in, scale_by_piv, out, cscale, st);
    if (!in_f64 && out_f64) return start_impl<float, uint16_t, float, double>(g, diag, piv, in, scale_by_piv, out, cscale, st);
    if (in_f64 && out_f64) return start_impl<float, uint16_t, double, double>(g, diag, piv, in, scale_by_piv, out, cscale, st);
    return start_impl<float, uint16_t, float, float>(g, diag, piv, in, scale_by_piv, out, cscale, st);
}

hipError_t launch_half_end(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                           bool in_f64, bool scale_by_piv, void *out, bool out_f64, hipStream_t st) {
    if (s == Store::F64) {
        if (!in_f64 || !out_f64) return hipErrorInvalidValue;
        return end_impl<double, double, double, double>(g, diag, piv, in, scale_by_piv, out, st);
    }
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return end_impl<float, float, double, float>(g, diag, piv, in, scale_by_piv, out, st);
        if (!in_f64 && !out_f64) return end_impl<float, float, float, float>(g, diag, piv, in, scale_by_piv, out, st);
        if (in_f64 && out_f64) return end_impl<float, float, double, double>(g, diag, piv, in, scale_by_piv, out, st);
        return end_impl<float, float, float, double>(g, diag, piv, in, scale_by_piv, out, st);
    }
    if (in_f64 && !out_f64) return end_impl<float, uint16_t, double, float>(g, diag, piv, in, scale_by_piv, out, st);
    if (!in_f64 && !out_f64) return end_impl<float, uint16_t, float, float>(g, diag, piv, in, scale_by_piv, out, st);
    if (in_f64 && out_f64) return end_impl<float, uint16_t, double, double>(g, diag, piv, in, scale_by_piv, out, st);
    return end_impl<float, uint16_t, float, double>(g, diag, piv, in, scale_by_piv, out, st);
}

hipError_t launch_ilu_pivots(const PassGeom &g, const double *const *diag, double *piv, int *bad, hipStream_t st) {
    PivArgs A{};
    A.g = g;
    for (int k = 0; k < 2 * g.dim + 1; ++k) A.diag[k] = diag[k];
    A.piv = piv;
    A.bad = bad;
    size_t sm = rings_bytes(g, sizeof(double));
    dim3 grid(g.ntiles), blk(block_threads(g));
    if (g.dim == 2)
        hipLaunchKernelGGL(k_ilu_pivots<2>, grid, blk, sm, st, A);
    else
        hipLaunchKernelGGL(k_ilu_pivots<3>, grid, blk, sm, st, A);
    return hipGetLastError();
}

// ------------------------------------------------------------------ vector kernels (FP64)
struct DiagPtrs {
    const double *d[7];
};
struct DiagOut {
    double *d[7];
};

__global__ void k_assemble(int dim, int n0, int n1, int n2, DiagPtrs al, double beta, DiagOut out) {
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int64_t m0 = n0 + 2, m1 = n1 + 2;
    for (int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; P < N; P += (int64_t)gridDim.x * blockDim.x) {
        int64_t x = P % n0, y = (P / n0) % n1, z = P / ((int64_t)n0 * n1);
        int64_t nd[3] = {x + 1, dim > 1 ? y + 1 : 0, dim > 2 ? z + 1 : 0};
        int64_t st[3] = {1, m0, m0 * m1};
        int64_t node = nd[0] + m0 * (nd[1] + m1 * nd[2]);
        double sum = 0.0;
        for (int a = 0; a < dim; ++a) {
            for (int s = -1; s <= 1; s += 2) {
                double ap = al.d[a][node], aq = al.d[a][node + s * st[a]];
                double face = 2.0 * ap * aq / (ap + aq);
                out.d[dk(a, s)][P] = face;
                sum += face;
            }
        }
        out.d[0][P] = sum + beta;
    }
}

template <int DIM>
__global__ void k_spmv(int n0, int n1, int n2, DiagPtrs D, const double *__restrict__ x, double *__restrict__ y,
                       const double *__restrict__ f) {
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    for (int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; P < N; P += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(P % n0);
        int j = (int)((P / n0) % n1);
        double acc = D.d[0][P] * x[P];
        if (i > 0) acc -= D.d[1][P] * x[P - 1];
        if (i < n0 - 1) acc -= D.d[2][P] * x[P + 1];
        if (j > 0) acc -= D.d[3][P] * x[P - s1];
        if (j < n1 - 1) acc -= D.d[4][P] * x[P + s1];
        if (DIM == 3) {
            int k = (int)(P / s2);
            if (k > 0) acc -= D.d[5][P] * x[P - s2];
            if (k < n2 - 1) acc -= D.d[6][P] * x[P + s2];
        }
        y[P] = f ? f[P] - acc : acc;
    }
}

// SpMV of a structurally symmetric operator stored as P, W, E, S, N (, B, F) diagonals whose
// lower couplings equal the upper couplings of the neighbours (a^W(P) = a^E(P - e_x), a^S(P) =
// a^N(P - e_y), a^B(P) = a^F(P - e_z)): the lower couplings are read as the neighbours' upper
// ones, the same values in the same order as k_spmv, so four (2D: three) diagonal streams
// come from HBM instead of seven (five); the shifted reads hit lines that neighbouring
// threads have just brought into the caches.
template <int DIM>
__global__ void k_spmv_sym(int n0, int n1, int n2, DiagPtrs D, const double *__restrict__ x, double *__restrict__ y) {
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    const double *__restrict__ aP = D.d[0], *__restrict__ aE = D.d[2], *__restrict__ aN = D.d[4];
    for (int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; P < N; P += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(P % n0);
        int j = (int)((P / n0) % n1);
        double acc = aP[P] * x[P];
        if (i > 0) acc -= aE[P - 1] * x[P - 1];
        if (i < n0 - 1) acc -= aE[P] * x[P + 1];
        if (j > 0) acc -= aN[P - s1] * x[P - s1];
        if (j < n1 - 1) acc -= aN[P] * x[P + s1];
        if (DIM == 3) {
            const double *__restrict__ aF = D.d[6];
            int k = (int)(P / s2);
            if (k > 0) acc -= aF[P - s2] * x[P - s2];
            if (k < n2 - 1) acc -= aF[P] * x[P + s2];
        }
        y[P] = acc;
    }
}

// flag[0] = 0 if some lower coupling differs (bit for bit) from the neighbour's upper coupling
__global__ void k_sym_check(int dim, int n0, int n1, int n2, DiagPtrs D, int *flag) {
    const int64_t N = (int64_t)n0 * n1 * n2;
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    bool ok = true;
    for (int64_t P = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; P < N; P += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(P % n0), j = (int)((P / n0) % n1);
        if (i < n0 - 1 && D.d[2][P] != D.d[1][P + 1]) ok = false;
        if (j < n1 - 1 && D.d[4][P] != D.d[3][P + s1]) ok = false;
        if (dim == 3) {
            const int k = (int)(P / s2);
            if (k < n2 - 1 && D.d[6][P] != D.d[5][P + s2]) ok = false;
        }
    }
    if (!ok) flag[0] = 0;
}

static unsigned grid_for(int64_t N, int threads = 256, int64_t cap = 8192) {
    int64_t b = (N + threads - 1) / threads;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_assemble(int dim, const int n[3], const double *const *alpha, double beta, double *const *diag,
                           hipStream_t st) {
    DiagPtrs al{};
    DiagOut out{};
    for (int a = 0; a < dim; ++a) al.d[a] = alpha[a];
    for (int k = 0; k < 2 * dim + 1; ++k) out.d[k] = diag[k];
    int64_t N = (int64_t)n[0] * n[1] * n[2];
    hipLaunchKernelGGL(k_assemble, dim3(grid_for(N)), dim3(256), 0, st, dim, n[0], n[1], n[2], al, beta, out);
    return hipGetLastError();
}

hipError_t launch_spmv(int dim, const int n[3], const double *const *diag, const double *x, double *y,
                       hipStream_t st) {
    DiagPtrs D{};
    for (int k = 0; k < 2 * dim + 1; ++k) D.d[k] = diag[k];
    int64_t N = (int64_t)n[0] * n[1] * n[2];
    if (dim == 2)
        hipLaunchKernelGGL(k_spmv<2>, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], n[2], D, x, y, (const double *)nullptr);
    else
        hipLaunchKernelGGL(k_spmv<3>, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], n[2], D, x, y, (const double *)nullptr);
    return hipGetLastError();
}

hipError_t launch_spmv_sym(int dim, const int n[3], const double *const *diag, const double *x, double *y,
                           hipStream_t st) {
    DiagPtrs D{};
    for (int k = 0; k < 2 * dim + 1; ++k) D.d[k] = diag[k];
    int64_t N = (int64_t)n[0] * n[1] * n[2];
    if (dim == 2)
        hipLaunchKernelGGL(k_spmv_sym<2>, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], n[2], D, x, y);
    else
        hipLaunchKernelGGL(k_spmv_sym<3>, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], n[2], D, x, y);
    return hipGetLastError();
}

hipError_t launch_sym_check(int dim, const int n[3], const double *const *diag, int *flag, hipStream_t st) {
    DiagPtrs D{};
    for (int k = 0; k < 2 * dim + 1; ++k) D.d[k] = diag[k];
    int64_t N = (int64_t)n[0] * n[1] * n[2];
    hipLaunchKernelGGL(k_sym_check, dim3(grid_for(N)), dim3(256), 0, st, dim, n[0], n[1], n[2], D, flag);
    return hipGetLastError();
}

hipError_t launch_residual(int dim, const int n[3], const double *const *diag, const double *f, const double *x,
                           double *r, hipStream_t st) {
    DiagPtrs D{};
    for (int k = 0; k < 2 * dim + 1; ++k) D.d[k] = diag[k];
    int64_t N = (int64_t)n[0] * n[1] * n[2];
    if (dim == 2)
        hipLaunchKernelGGL(k_spmv<2>, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], n[2], D, x, r, f);
    else
        hipLaunchKernelGGL(k_spmv<3>, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], n[2], D, x, r, f);
    return hipGetLastError();
}

// ---------------------------------------------------------------- stationary sweep as a start-coupled pass
// One decomposed SOR sweep in direction map g.sig (Secs. 2-4) multiplied by a^P/omega is
//   (a^P/w - N1) u_new = f + (1/w - 1) a^P u_old + N2 u_old ,
// w the factor of the point's own subdomain's start corner, N1 / N2 the couplings towards the
// upstream / downstream neighbours (whatever subdomain owns them).  The right-hand side below and
// the pivots a^P/w, per point, turn the sweep into a start-coupled half-sweep of the pipelined kind.

// subdomain coordinate of global coordinate x on an axis of n points cut into p ranges, the first
// n mod p of them one point longer
__device__ __forceinline__ int part_of(int x, int n, int p) {
    const int base = n / p, rem = n % p, big = rem * (base + 1);
    return x < big ? x / (base + 1) : rem + (x - big) / base;
}

struct Omega8 {
    double w[8];
};

__global__ void k_sor_rhs2d(int n0, int n1, int p0, int p1, int sig0, int sig1, DiagPtrs D, Omega8 om,
                            const double *__restrict__ f, const double *__restrict__ uold, double *__restrict__ out) {
    const int64_t N = (int64_t)n0 * n1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % n0), y = (int)(i / n0);
        const int d0 = (part_of(x, n0, p0) & 1) ? -sig0 : sig0;
        const int d1 = (part_of(y, n1, p1) & 1) ? -sig1 : sig1;
        const int c = (d0 < 0 ? 1 : 0) | (d1 < 0 ? 2 : 0);
        const double w = c == 0 ? om.w[0] : c == 1 ? om.w[1] : c == 2 ? om.w[2] : om.w[3];
        const double aP = D.d[0][i];
        double acc = f[i] + (1.0 / w - 1.0) * aP * uold[i];
        // downstream neighbours: the side the point's own sweep moves towards
        const int xd = x + d0, yd = y + d1;
        if (xd >= 0 && xd < n0) acc += D.d[d0 > 0 ? 2 : 1][i] * uold[i + d0];
        if (yd >= 0 && yd < n1) acc += D.d[d1 > 0 ? 4 : 3][i] * uold[i + (int64_t)d1 * n0];
        out[i] = acc;
    }
}

__global__ void k_sor_piv2d(int n0, int n1, int p0, int p1, int sig0, int sig1, const double *__restrict__ aP,
                            Omega8 om, double *__restrict__ piv) {
    const int64_t N = (int64_t)n0 * n1;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(i % n0), y = (int)(i / n0);
        const int d0 = (part_of(x, n0, p0) & 1) ? -sig0 : sig0;
        const int d1 = (part_of(y, n1, p1) & 1) ? -sig1 : sig1;
        const int c = (d0 < 0 ? 1 : 0) | (d1 < 0 ? 2 : 0);
        piv[i] = aP[i] / (c == 0 ? om.w[0] : c == 1 ? om.w[1] : c == 2 ? om.w[2] : om.w[3]);
    }
}

// FP64 -> storage precision (FP32: the hardware's round to nearest even; BF16: f64_to_bf16)
__global__ void k_convert(const double *src, void *dst, int kind, int64_t N, double scale) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double v = src[i] * scale;
        if (kind == 0) ((double *)dst)[i] = v;
        else if (kind == 1) ((float *)dst)[i] = (float)v;
        else ((uint16_t *)dst)[i] = f64_to_bf16(v);
    }
}

hipError_t launch_sor_rhs2d(const int n[3], const int p[3], const int sig[3], const double *const *diag,
                           const double *omega8, const double *f, const double *uold, double *out, hipStream_t st) {
    DiagPtrs D{};
    for (int k = 0; k < 5; ++k) D.d[k] = diag[k];
    Omega8 om{};
    for (int k = 0; k < 8; ++k) om.w[k] = omega8[k];
    const int64_t N = (int64_t)n[0] * n[1];
    hipLaunchKernelGGL(k_sor_rhs2d, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], p[0], p[1], sig[0], sig[1], D,
                       om, f, uold, out);
    return hipGetLastError();
}

hipError_t launch_sor_piv2d(const int n[3], const int p[3], const int sig[3], const double *aP, const double *omega8,
                            double *piv, hipStream_t st) {
    Omega8 om{};
    for (int k = 0; k < 8; ++k) om.w[k] = omega8[k];
    const int64_t N = (int64_t)n[0] * n[1];
    hipLaunchKernelGGL(k_sor_piv2d, dim3(grid_for(N)), dim3(256), 0, st, n[0], n[1], p[0], p[1], sig[0], sig[1], aP,
                       om, piv);
    return hipGetLastError();
}

hipError_t launch_convert(const double *src, void *dst, Store s, int64_t N, double scale, hipStream_t st) {
    hipLaunchKernelGGL(k_convert, dim3(grid_for(N)), dim3(256), 0, st, src, dst, (int)s, N, scale);
    return hipGetLastError();
}

__global__ void k_scale_add(double *z, const double *a, double ca, const void *b, int b_f64, double cb, int64_t N) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double bv = b ? (b_f64 ? ((const double *)b)[i] : (double)((const float *)b)[i]) : 0.0;
        double av = a ? a[i] : 0.0;
        z[i] = ca * av + cb * bv;
    }
}

hipError_t launch_scale_add(double *z, const double *a, double ca, const void *b, bool b_f64, double cb, int64_t N,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_scale_add, dim3(grid_for(N)), dim3(256), 0, st, z, a, ca, b, b_f64 ? 1 : 0, cb, N);
    return hipGetLastError();
}

// deterministic block reduction of one value per thread (fixed tree)
__device__ __forceinline__ double block_sum(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kRedThreads) k_dot_partial(const double *x, const double *y, int64_t N, double *partials) {
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    const int64_t stride = (int64_t)kRedBlocks * kRedThreads;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < N; i += stride) acc += x[i] * y[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// sums `groups` consecutive groups of kRedBlocks partials; out[g] per group
__global__ void __launch_bounds__(kRedThreads) k_dot_final(const double *partials, double *out) {
    __shared__ double sh[kRedThreads];
    const double *p = partials + (int64_t)blockIdx.x * kRedBlocks;
    double acc = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += kRedThreads) acc += p[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

hipError_t launch_dot(const double *x, const double *y, int64_t N, double *partials, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, st, x, y, N, partials);
    hipLaunchKernelGGL(k_dot_final, dim3(1), dim3(kRedThreads), 0, st, partials, out);
    return hipGetLastError();
}

hipError_t launch_dot_partial(const double *x, const double *y, int64_t N, double *partials, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(kRedThreads), 0, st, x, y, N, partials);
    return hipGetLastError();
}

// 3D q = A x (7-point), the Krylov operator product outside the fused CG step.  Each thread walks
// one (x, y) column through a run of z planes and keeps the values of the planes below and above in
// registers, so x and the z couplings come from HBM once; the in-plane neighbours hit lines that
// the neighbouring lanes and waves load for their own columns.  Every load is unconditional
// (clamped index; an absent neighbour gets a zero coupling), and so is the store: a lane past the
// grid's edge works on the clamped edge column and writes the same bits as that column's own lane,
// so no load is sunk under a branch and waits there.  The terms are taken in the order of k_spmv.
// SYM: the lower couplings are the neighbours' upper ones (a^W(P) = a^E(P - e_x), a^S(P) =
// a^N(P - e_y), a^B(P) = a^F(P - e_z)).  Blocks walk (column tile, z run) items; with a block count
// that is a multiple of 8, block b starts at item (b mod 8) * (blocks / 8) + b / 8, so the blocks
// of one XCD (b mod 8) hold neighbouring tiles of one z run and meet each other's halo lines in
// their L2.
constexpr int kSp3X = 64, kSp3Y = 4;

template <bool SYM>
__global__ void __launch_bounds__(kSp3X *kSp3Y)
    k_spmv3(int n0, int n1, int n2, int ntx, int nty, int lz, int nitems, DiagPtrs D, const double *__restrict__ x,
            double *__restrict__ q) {
    const int nb = gridDim.x, b = blockIdx.x;
    const int start = (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
    const int64_t s1 = n0, s2 = (int64_t)n0 * n1;
    const int lx = threadIdx.x % kSp3X, ly = threadIdx.x / kSp3X;
    const double *__restrict__ aP = D.d[0], *__restrict__ aE = D.d[2], *__restrict__ aN = D.d[4];
    const double *__restrict__ aF = D.d[6];
    for (int it = start; it < nitems; it += nb) {
        const int cx = it % ntx, rest = it / ntx, cy = rest % nty, cz = rest / nty;
        const int i = cx * kSp3X + lx, j = cy * kSp3Y + ly;
        const int ic = min(i, n0 - 1), jc = min(j, n1 - 1);
        const int k0 = cz * lz, k1 = min(n2, k0 + lz);
        const bool hw = ic > 0, he = ic < n0 - 1, hs = jc > 0, hn = jc < n1 - 1;
        const int oW = hw ? -1 : 0, oE = he ? 1 : 0, oS = hs ? -n0 : 0, oN = hn ? n0 : 0;
        int64_t P = ic + (int64_t)jc * s1 + (int64_t)k0 * s2;
        const int64_t Pb = k0 > 0 ? P - s2 : P;
        double xb = x[Pb];                   // x of the plane below
        double cb = SYM ? aF[Pb] : 0.0;      // (SYM) its upper z coupling = this point's a^B
        double xc = x[P];
        for (int k = k0; k < k1; ++k, P += s2) {
            const bool hu = k < n2 - 1, hd = k > 0;
            const double xu = x[hu ? P + s2 : P];
            const double cP = aP[P];
            const double cW = SYM ? aE[P + oW] : D.d[1][P];
            const double cE = aE[P];
            const double cS = SYM ? aN[P + oS] : D.d[3][P];
            const double cN = aN[P];
            const double cB = SYM ? cb : D.d[5][P];
            const double cF = aF[P];
            const double xW = x[P + oW], xE = x[P + oE], xS = x[P + oS], xN = x[P + oN];
            double acc = cP * xc;
            acc = fma(-(hw ? cW : 0.0), xW, acc);
            acc = fma(-(he ? cE : 0.0), xE, acc);
            acc = fma(-(hs ? cS : 0.0), xS, acc);
            acc = fma(-(hn ? cN : 0.0), xN, acc);
            acc = fma(-(hd ? cB : 0.0), xb, acc);
            acc = fma(-(hu ? cF : 0.0), xu, acc);
            q[P] = acc;
            xb = xc;
            xc = xu;
            cb = cF;
        }
    }
}

// Items of k_spmv3: column tiles of kSp3X x kSp3Y, each cut into z runs of lz
// planes when the tiles alone are fewer than kRedBlocks; blocks = min(items, kRedBlocks).
struct Sp3Plan {
    int ntx, nty, lz, items, nb;
};

static bool sp3_plan(const int n[3], Sp3Plan &pl) {
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) return false;
    pl.ntx = (n[0] + kSp3X - 1) / kSp3X;
    pl.nty = (n[1] + kSp3Y - 1) / kSp3Y;
    const int64_t ncol = (int64_t)pl.ntx * pl.nty;
    int nz = ncol < kRedBlocks ? (int)std::min<int64_t>(n[2], kRedBlocks / ncol) : 1;
    pl.lz = (n[2] + nz - 1) / nz;
    nz = (n[2] + pl.lz - 1) / pl.lz;
    const int64_t items = ncol * nz;
    if (items > (int64_t)0x7fffffff) return false;
    pl.items = (int)items;
    pl.nb = (int)std::min<int64_t>(items, kRedBlocks);
    return true;
}

hipError_t launch_spmv3(const int n[3], const double *const *diag, bool sym, const double *x, double *q,
                        hipStream_t st) {
    Sp3Plan pl;
    if (!sp3_plan(n, pl)) return hipErrorInvalidValue;
    DiagPtrs D{};
    for (int k = 0; k < 7; ++k) D.d[k] = diag[k];
    if (sym)
        hipLaunchKernelGGL(k_spmv3<true>, dim3(pl.nb), dim3(kSp3X * kSp3Y), 0, st, n[0], n[1], n[2], pl.ntx,
                           pl.nty, pl.lz, pl.items, D, x, q);
    else
        hipLaunchKernelGGL(k_spmv3<false>, dim3(pl.nb), dim3(kSp3X * kSp3Y), 0, st, n[0], n[1], n[2], pl.ntx,
                           pl.nty, pl.lz, pl.items, D, x, q);
    return hipGetLastError();
}

// z = 0.5 z1 + b z2, with one rounding after the exact halving (the symmetric preconditioner's combination)
__device__ __forceinline__ double zcomb(double z1, double z2, double b) { return __fma_rn(b, z2, 0.5 * z1); }

template <typename Z2>
__global__ void __launch_bounds__(kRedThreads) k_dot_partial_zz(const double *r, const double *z1, const Z2 *z2,
                                                               double b, int64_t N, double *partials) {
    __shared__ double sh[kRedThreads];
    double acc = 0.0;
    const int64_t stride = (int64_t)kRedBlocks * kRedThreads;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < N; i += stride)
        acc += r[i] * zcomb(z1[i], (double)z2[i], b);
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

hipError_t launch_dot_partial_zz(const double *r, const double *z1, const double *z2, double b, int64_t N,
                                 double *partials, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial_zz<double>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, r, z1, z2, b, N, partials);
    return hipGetLastError();
}

// the same with the second piece in FP32 (the output of FP32/BF16 sweeps)
hipError_t launch_dot_partial_zf(const double *r, const double *z1, const float *z2, double b, int64_t N,
                                 double *partials, hipStream_t st) {
    hipLaunchKernelGGL(k_dot_partial_zz<float>, dim3(kRedBlocks), dim3(kRedThreads), 0, st, r, z1, z2, b, N, partials);
    return hipGetLastError();
}

// ------------------------------------------------ fused CG step, 5-point operator
// Lane l takes lane l-1's value (lane 0: 0), or lane l+1's value (lane 63: 0):
// DPP wave shifts, 32 bits at a time, all lanes active.
__device__ __forceinline__ double from_lower_lane(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_upper_lane(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x130, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x130, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum of n partials in a fixed order by one wave (lane-strided, then an xor
// butterfly); every lane of every wave obtains the same value, with no barrier.
__device__ __forceinline__ double wave_sum_partials(const double *p, int n) {
    double acc = 0.0;
    for (int i = (int)(threadIdx.x & 63); i < n; i += 64) acc += p[i];
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    return acc;
}

// streaming (nontemporal) loads of one or two doubles for the 2D fused CG step: its streams are
// read once, and without the hint their lines push the next passes' coefficients out of the caches
template <int V>
__device__ __forceinline__ void ldv(const double *__restrict__ a, int64_t P, double (&o)[V]) {
    if constexpr (V == 2) {
        typedef double ntl_d2 __attribute__((ext_vector_type(2)));
        const ntl_d2 t = __builtin_nontemporal_load(reinterpret_cast<const ntl_d2 *>(a + P));
        o[0] = t.x;
        o[1] = t.y;
    } else {
        o[0] = __builtin_nontemporal_load(a + P);
    }
}
// streaming (nontemporal) stores of one or two doubles: lines written by a pass over the grid and
// not read again by it, so that they do not take L2 room from the lines it still reads
typedef double nt_d2 __attribute__((ext_vector_type(2)));
template <int V> __device__ __forceinline__ void stv(double *__restrict__ a, int64_t P, const double (&v)[V]) {
    if constexpr (V == 2) {
        nt_d2 t = {v[0], v[1]};
        __builtin_nontemporal_store(t, reinterpret_cast<nt_d2 *>(a + P));
    } else
        __builtin_nontemporal_store(v[0], a + P);
}

// inputs of the new p on one row (z pieces, old p) and the operator row with x
template <int V> struct CgRowIn {
    double z1[V], z2[V], po[V];
};
template <int V> struct CgRowOp {
    double d[5][V], x[V];
};

// One CG step on a 2D grid, fused over tiles of kCgRows rows by 256 V columns
// (V = 2 columns per lane where rows are 16-byte aligned):
//   beta = rz / rz_old (rz from its partials; 0 on the first step), p = z + beta p_old,
//   x += alpha_prev p_old (the previous step's update, deferred), q = A p,
//   and the block's partial of p.q.
// z = zcomb(z1, z2, hb) in the split form of the symmetric preconditioner, else z1.
// p goes to a second buffer, so every thread forms the new p of its neighbours
// from their old p: inside a wave by lane shifts, the rows above and below slide
// through registers (read two rows ahead), and the column beyond each side of
// the wave is formed once per tile by a gather and handed out row by row.
// The blocks of one XCD (blockIdx mod 8) take one contiguous range of tiles,
// so vertically adjacent tiles, and their halo rows, share that XCD's L2.
// SYM: symmetric storage (checked at set-up): the W coupling of a point is the E coupling of its
// left neighbour (the lane to the left, or the wave's left halo column gathered per tile) and the
// S coupling the N coupling of the row below (carried from the previous row): three diagonal
// streams instead of five, the same values in the same order.
constexpr int kCgRows = 16;
template <bool SPLIT, int V, bool SYM>
__global__ void __launch_bounds__(256) k_cg_pq2d(int n0, int n1, int nbx, int ntiles, int tpb, DiagPtrs D,
                                                 const double *__restrict__ z1, const double *__restrict__ z2,
                                                 double hb, const double *__restrict__ pold, double *__restrict__ pnew,
                                                 double *__restrict__ q, double *__restrict__ x, const double *rz_part,
                                                 double *rz_new, const double *rz_old, const double *alpha_prev,
                                                 int first, double *pq_part) {
    __shared__ double sh[256];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const double rz = wave_sum_partials(rz_part, kRedBlocks);
    if (blockIdx.x == 0 && threadIdx.x == 0) rz_new[0] = rz;
    const double beta = first ? 0.0 : rz / rz_old[0];
    const double alpha = first ? 0.0 : alpha_prev[0];
    auto newp = [&](double a1, double a2, double po) {
        const double z = SPLIT ? zcomb(a1, a2, hb) : a1;
        return first ? z : __fma_rn(beta, po, z);
    };
    auto load_in = [&](CgRowIn<V> &r, int64_t P) {
        ldv<V>(z1, P, r.z1);
        if (SPLIT) ldv<V>(z2, P, r.z2);
        if (!first) ldv<V>(pold, P, r.po);
    };
    auto load_op = [&](CgRowOp<V> &o, int64_t P) {
#pragma unroll
        for (int k = 0; k < 5; ++k)
            if (!SYM || k % 2 == 0) ldv<V>(D.d[k], P, o.d[k]);
        if (!first) ldv<V>(x, P, o.x);
    };
    auto form = [&](const CgRowIn<V> &r, double (&o)[V]) {
#pragma unroll
        for (int c = 0; c < V; ++c) o[c] = newp(r.z1[c], SPLIT ? r.z2[c] : 0.0, first ? 0.0 : r.po[c]);
    };
    const int G = gridDim.x;
    const int vb = (int)(blockIdx.x & 7) * (G >> 3) + (int)(blockIdx.x >> 3);
    const int t0 = vb * tpb, t1 = min(t0 + tpb, ntiles);
    double acc = 0.0;
    for (int t = t0; t < t1; ++t) {
        const int c0 = (t % nbx) * (256 * V) + wave * (64 * V); // the wave's first column
        const int i = c0 + lane * V;
        const int j0 = (t / nbx) * kCgRows, j1 = min(j0 + kCgRows, n1);
        const bool in = i < n0;
        const int ic = in ? i : 0; // loads of lanes beyond the grid read column 0 and are dropped
        // new p on the columns beyond the wave's two sides, rows j0-1 .. j1: lanes 0.. left, 32.. right
        double hn = 0.0, he = 0.0; // he (SYM, left column): its E coupling, the W of column c0
        {
            const int hr = lane & 31, hrow = j0 - 1 + hr;
            const int hcol = (lane >> 5) ? c0 + 64 * V : c0 - 1;
            if (hr < j1 - j0 + 2 && hrow >= 0 && hrow < n1 && hcol >= 0 && hcol < n0) {
                const int64_t H = (int64_t)hrow * n0 + hcol;
                hn = newp(z1[H], SPLIT ? z2[H] : 0.0, first ? 0.0 : pold[H]);
                if (SYM && !(lane >> 5)) he = D.d[2][H];
            }
        }
        // SYM: the N coupling of the row below the strip (the S coupling of its first row)
        double nprev[V];
#pragma unroll
        for (int c = 0; c < V; ++c) nprev[c] = 0.0;
        if (SYM && j0 > 0) ldv<V>(D.d[4], (int64_t)(j0 - 1) * n0 + ic, nprev);
        double pm[V], pc[V], oc[V];
        CgRowIn<V> ra, rb; // new-p inputs of rows j+1 and j+2
        CgRowOp<V> oa, ob; // operator rows j and j+1
        {
            CgRowIn<V> r;
            load_in(r, (int64_t)max(j0 - 1, 0) * n0 + ic);
            form(r, pm);
            load_in(r, (int64_t)j0 * n0 + ic);
            form(r, pc);
#pragma unroll
            for (int c = 0; c < V; ++c) oc[c] = first ? 0.0 : r.po[c];
        }
        load_in(ra, (int64_t)min(j0 + 1, n1 - 1) * n0 + ic);
        load_op(oa, (int64_t)j0 * n0 + ic);
        for (int j = j0; j < j1; ++j) {
            // read ahead, but never past what the strip uses (the new p of row j1, the operator of row j1 - 1):
            // the clamped loads re-read a row already in cache
            load_in(rb, (int64_t)min(j + 2, min(j1, n1 - 1)) * n0 + ic);
            load_op(ob, (int64_t)min(j + 1, j1 - 1) * n0 + ic);
            double pp[V];
            form(ra, pp);
            const double sl = from_lower_lane(pc[V - 1]), sr = from_upper_lane(pc[0]); // every lane takes part
            const double h = __shfl(hn, (lane == 63 ? 32 : 0) + (j - j0 + 1), 64);
            double wc[V], sc[V]; // W and S couplings of this row
            if (SYM) {
                const double el = from_lower_lane(oa.d[2][V - 1]);
                const double eh = __shfl(he, j - j0 + 1, 64);
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    wc[c] = c > 0 ? oa.d[2][c - 1] : (lane == 0 ? eh : el);
                    sc[c] = nprev[c];
                }
            } else {
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    wc[c] = oa.d[1][c];
                    sc[c] = oa.d[3][c];
                }
            }
            if (in) {
                const int64_t P = (int64_t)j * n0 + i;
                double qa[V], xn[V];
#pragma unroll
                for (int c = 0; c < V; ++c) {
                    const double pl = c > 0 ? pc[c - 1] : (lane == 0 ? h : sl);
                    const double pr = c < V - 1 ? pc[c + 1] : (lane == 63 ? h : sr);
                    double a = oa.d[0][c] * pc[c];
                    if (i + c > 0) a -= wc[c] * pl;
                    if (i + c < n0 - 1) a -= oa.d[2][c] * pr;
                    if (j > 0) a -= sc[c] * pm[c];
                    if (j < n1 - 1) a -= oa.d[4][c] * pp[c];
                    qa[c] = a;
                    acc += pc[c] * a;
                    xn[c] = first ? 0.0 : oa.x[c] + alpha * oc[c];
                }
                stv<V>(q, P, qa);
                stv<V>(pnew, P, pc);
                if (!first) stv<V>(x, P, xn);
            }
#pragma unroll
            for (int c = 0; c < V; ++c) {
                pm[c] = pc[c];
                pc[c] = pp[c];
                oc[c] = first ? 0.0 : ra.po[c];
                nprev[c] = oa.d[4][c];
            }
            ra = rb;
            oa = ob;
        }
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) pq_part[blockIdx.x] = s;
}

hipError_t launch_cg_pq2d(int n0, int n1, const double *const *diag, const double *z1, const double *z2, double hb,
                          const double *pold, double *pnew, double *q, double *x, const double *rz_part,
                          double *rz_new, const double *rz_old, const double *alpha_prev, bool first,
                          double *pq_part, int *npq, bool sym, hipStream_t st) {
    DiagPtrs D{};
    bool al = n0 % 2 == 0;
    for (int k = 0; k < 5; ++k) {
        D.d[k] = diag[k];
        al = al && ((uintptr_t)diag[k] & 15) == 0;
    }
    for (const void *ptr : {(const void *)z1, (const void *)z2, (const void *)pold, (const void *)pnew,
                            (const void *)q, (const void *)x})
        al = al && ((uintptr_t)ptr & 15) == 0;
    const int V = al ? 2 : 1;
    const int nbx = (n0 + 256 * V - 1) / (256 * V), nby = (n1 + kCgRows - 1) / kCgRows;
    const int ntiles = nbx * nby;
    int grid = std::min(ntiles, kRedBlocks);
    grid = (grid + 7) / 8 * 8; // at most kRedBlocks, a multiple of 8
    *npq = grid;
    const int tpb = (ntiles + grid - 1) / grid;
#define PSW_CG_PQ(S, VV, SY)                                                                                          \
    hipLaunchKernelGGL((k_cg_pq2d<S, VV, SY>), dim3(grid), dim3(256), 0, st, n0, n1, nbx, ntiles, tpb, D, z1, z2, hb,\
                       pold, pnew, q, x, rz_part, rz_new, rz_old, alpha_prev, (int)first, pq_part)
    if (sym) {
        if (z2) {
            if (V == 2) PSW_CG_PQ(true, 2, true); else PSW_CG_PQ(true, 1, true);
        } else {
            if (V == 2) PSW_CG_PQ(false, 2, true); else PSW_CG_PQ(false, 1, true);
        }
    } else if (z2) {
        if (V == 2) PSW_CG_PQ(true, 2, false); else PSW_CG_PQ(true, 1, false);
    } else {
        if (V == 2) PSW_CG_PQ(false, 2, false); else PSW_CG_PQ(false, 1, false);
    }
#undef PSW_CG_PQ
    return hipGetLastError();
}

// ------------------------------------------------ fused CG step, 7-point operator
// Element i of an array: with 32-bit indices (I = uint32_t, used when every byte offset fits in
// 31 bits) the byte offset is formed in 32 bits, so the loads take an SGPR base and one VGPR
// offset instead of a 64-bit address per load.
template <typename I, typename T> __device__ __forceinline__ const T &elt(const T *b, I i) {
    if constexpr (sizeof(I) == 4)
        return *reinterpret_cast<const T *>(reinterpret_cast<const char *>(b) + (uint32_t)(i * (uint32_t)sizeof(T)));
    else
        return b[i];
}
template <typename I, typename T> __device__ __forceinline__ T &elt(T *b, I i) {
    if constexpr (sizeof(I) == 4)
        return *reinterpret_cast<T *>(reinterpret_cast<char *>(b) + (uint32_t)(i * (uint32_t)sizeof(T)));
    else
        return b[i];
}

// The 3D counterpart of k_cg_pq2d: beta = rz / rz_old[0] with rz the sum of kRedBlocks partials
// (stored to rz_new[0]; beta = 0 when first), pnew = z + beta pold with z = 0.5 z1 + hb z2
// (SPLIT: z2 the FP32 piece of the split preconditioner) or z = z1, x += alpha_prev[0] pold (not
// when first), q = A pnew, and one partial of pnew.q per block (*npq of them).  The columns march
// through z runs as in k_spmv3: pnew of the planes below and above stays in registers, and each
// in-plane neighbour's pnew is formed again from its z and pold (lines that the neighbouring lanes
// and waves load for their own columns), so no point waits for another's result.  Each step issues
// all its loads before the first use.  pnew and q are stored by every lane (a lane past the grid's
// edge stores its clamped column's bits again); x, read and written, only by the column's own lane.
template <bool SYM, bool SPLIT, typename I>
__global__ void __launch_bounds__(kSp3X *kSp3Y)
    k_cg_pq3d(int n0, int n1, int n2, int ntx, int nty, int lz, int nitems, DiagPtrs D,
              const double *__restrict__ z1, const float *__restrict__ z2, double hb,
              const double *__restrict__ pold, double *__restrict__ pnew, double *__restrict__ q,
              double *__restrict__ x, const double *rz_part, double *rz_new, const double *rz_old,
              const double *alpha_prev, int first, double *pq_part) {
    __shared__ double sh[kSp3X * kSp3Y];
    __shared__ double s_rz;
    if (threadIdx.x < 64) {
        const double v = wave_sum_partials(rz_part, kRedBlocks);
        if (threadIdx.x == 0) s_rz = v;
    }
    __syncthreads();
    const double rz = s_rz;
    if (blockIdx.x == 0 && threadIdx.x == 0) rz_new[0] = rz;
    const double beta = first ? 0.0 : rz / rz_old[0];
    const double alpha = first ? 0.0 : alpha_prev[0];
    // pnew from z1, z2 and pold at one point (pold read also when first, and then not used)
    auto form = [&](double a1, float a2, double po) -> double {
        const double zv = SPLIT ? zcomb(a1, (double)a2, hb) : a1;
        return first ? zv : __fma_rn(beta, po, zv);
    };
    const int nb = gridDim.x, b = blockIdx.x;
    const int start = (nb & 7) == 0 ? (b & 7) * (nb >> 3) + (b >> 3) : b;
    const I s1 = (I)n0, s2 = (I)n0 * (I)n1;
    const int lx = threadIdx.x % kSp3X, ly = threadIdx.x / kSp3X;
    const double *__restrict__ aP = D.d[0], *__restrict__ aE = D.d[2], *__restrict__ aN = D.d[4];
    const double *__restrict__ aF = D.d[6];
    double dot = 0.0;
    for (int it = start; it < nitems; it += nb) {
        const int cx = it % ntx, rest = it / ntx, cy = rest % nty, cz = rest / nty;
        const int i = cx * kSp3X + lx, j = cy * kSp3Y + ly;
        const bool own = i < n0 && j < n1;
        const int ic = min(i, n0 - 1), jc = min(j, n1 - 1);
        const int k0 = cz * lz, k1 = min(n2, k0 + lz);
        const bool hw = ic > 0, he = ic < n0 - 1, hs = jc > 0, hn = jc < n1 - 1;
        const I oW = hw ? (I)-1 : (I)0, oE = he ? (I)1 : (I)0, oS = hs ? (I)0 - s1 : (I)0, oN = hn ? s1 : (I)0;
        I P = (I)ic + (I)jc * s1 + (I)k0 * s2;
        const I Pb = k0 > 0 ? P - s2 : P;
        double pb = form(elt(z1, Pb), SPLIT ? elt(z2, Pb) : 0.f, elt(pold, Pb)); // pnew of the plane below
        double cb = SYM ? elt(aF, Pb) : 0.0; // (SYM) its upper z coupling = this point's a^B
        double poc = elt(pold, P);
        double pc = form(elt(z1, P), SPLIT ? elt(z2, P) : 0.f, poc);
        // the run's first values are waited for here, once, and not at every step's head
        __asm__ volatile("" : : "v"(pb), "v"(cb), "v"(poc), "v"(pc));
        for (int k = k0; k < k1; ++k, P += s2) {
            const bool hu = k < n2 - 1, hd = k > 0;
            // every load of the step is issued before the first use (order: the plane above,
            // the four in-plane neighbours, the couplings, x last)
            const I Q[5] = {hu ? P + s2 : P, P + oW, P + oE, P + oS, P + oN};
            double l1[5], lo[5];
            float l2[5];
#pragma unroll
            for (int u = 0; u < 5; ++u) {
                l1[u] = elt(z1, Q[u]);
                l2[u] = SPLIT ? elt(z2, Q[u]) : 0.f;
                lo[u] = elt(pold, Q[u]);
            }
            // a^P, a^F and x are read once, by this point's lane: streaming loads
            const double cP = __builtin_nontemporal_load(&elt(aP, P));
            const double cW = SYM ? elt(aE, P + oW) : elt(D.d[1], P);
            const double cE = elt(aE, P);
            const double cS = SYM ? elt(aN, P + oS) : elt(D.d[3], P);
            const double cN = elt(aN, P);
            const double cB = SYM ? cb : elt(D.d[5], P);
            const double cF = __builtin_nontemporal_load(&elt(aF, P));
            const double xv = __builtin_nontemporal_load(&elt((const double *)x, P));
            __builtin_amdgcn_sched_barrier(0);
            double pn[5];
#pragma unroll
            for (int u = 0; u < 5; ++u) pn[u] = form(l1[u], l2[u], lo[u]);
            double acc = cP * pc;
            acc = fma(-(hw ? cW : 0.0), pn[1], acc);
            acc = fma(-(he ? cE : 0.0), pn[2], acc);
            acc = fma(-(hs ? cS : 0.0), pn[3], acc);
            acc = fma(-(hn ? cN : 0.0), pn[4], acc);
            acc = fma(-(hd ? cB : 0.0), pb, acc);
            acc = fma(-(hu ? cF : 0.0), pn[0], acc);
            // streaming stores: the written lines are not read again in this kernel, and the
            // neighbours' lines it does read stay in L2 (measured 1.3 % per 256^3 solve)
            __builtin_nontemporal_store(pc, &elt(pnew, P));
            __builtin_nontemporal_store(acc, &elt(q, P));
            dot = fma(own ? pc : 0.0, acc, dot);
            // xv is used here, outside the branch, so that its load stays with the others
            // instead of being moved under the branch and waited for there
            __asm__ volatile("" : : "v"(xv));
            if (own && !first) __builtin_nontemporal_store(__fma_rn(alpha, poc, xv), &elt(x, P));
            pb = pc;
            pc = pn[0];
            poc = lo[0];
            cb = cF;
        }
    }
    const double s = block_sum(dot, sh);
    if (threadIdx.x == 0) pq_part[b] = s;
}

// blocks of k_cg_pq3d<SYM, SPLIT, I> resident on the device at once (queried once per instance)
template <bool SYM, bool SPLIT, typename I> static int cg_pq3d_resident() {
    static int cached = 0;
    if (cached == 0) {
        int dev = 0, ncu = 0, per = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_cg_pq3d<SYM, SPLIT, I>, kSp3X * kSp3Y, 0) !=
                hipSuccess || ncu < 1 || per < 1)
            return kRedBlocks;
        cached = std::min(ncu * per, kCgPq3dMaxBlocks);
    }
    return cached;
}

template <bool SYM, bool SPLIT, typename I>
static hipError_t cg_pq3d_launch(const int n[3], const DiagPtrs &D, const double *z1, const float *z2, double hb,
                                 const double *pold, double *pnew, double *q, double *x, const double *rz_part,
                                 double *rz_new, const double *rz_old, const double *alpha_prev, bool first,
                                 double *pq_part, int *npq, hipStream_t st) {
    // one z run per resident block where the column tiles allow it, so the blocks run in one round
    const int cap = cg_pq3d_resident<SYM, SPLIT, I>();
    const int ntx = (n[0] + kSp3X - 1) / kSp3X, nty = (n[1] + kSp3Y - 1) / kSp3Y;
    const int64_t ncol = (int64_t)ntx * nty;
    int nz = ncol < cap ? (int)std::min<int64_t>(n[2], cap / ncol) : 1;
    const int lz = (n[2] + nz - 1) / nz;
    nz = (n[2] + lz - 1) / lz;
    const int64_t items = ncol * nz;
    if (items > (int64_t)0x7fffffff) return hipErrorInvalidValue;
    const int nb = (int)std::min<int64_t>(items, cap);
    *npq = nb;
    hipLaunchKernelGGL((k_cg_pq3d<SYM, SPLIT, I>), dim3(nb), dim3(kSp3X * kSp3Y), 0, st, n[0], n[1], n[2], ntx, nty,
                       lz, (int)items, D, z1, z2, hb, pold, pnew, q, x, rz_part, rz_new, rz_old, alpha_prev,
                       (int)first, pq_part);
    return hipGetLastError();
}

hipError_t launch_cg_pq3d(const int n[3], const double *const *diag, const double *z1, const float *z2, double hb,
                          const double *pold, double *pnew, double *q, double *x, const double *rz_part,
                          double *rz_new, const double *rz_old, const double *alpha_prev, bool first,
                          double *pq_part, int *npq, bool sym, hipStream_t st) {
    if (n[0] < 1 || n[1] < 1 || n[2] < 1) return hipErrorInvalidValue;
    DiagPtrs D{};
    for (int k = 0; k < 7; ++k) D.d[k] = diag[k];
    const bool i32 = (int64_t)n[0] * n[1] * n[2] * (int64_t)sizeof(double) < ((int64_t)1 << 31);
#define PSW_CG_PQ3(SY, SP)                                                                                           \
    (i32 ? cg_pq3d_launch<SY, SP, uint32_t>(n, D, z1, z2, hb, pold, pnew, q, x, rz_part, rz_new, rz_old,            \
                                            alpha_prev, first, pq_part, npq, st)                                     \
         : cg_pq3d_launch<SY, SP, int64_t>(n, D, z1, z2, hb, pold, pnew, q, x, rz_part, rz_new, rz_old,             \
                                           alpha_prev, first, pq_part, npq, st))
    hipError_t e;
    if (sym)
        e = z2 ? PSW_CG_PQ3(true, true) : PSW_CG_PQ3(true, false);
    else
        e = z2 ? PSW_CG_PQ3(false, true) : PSW_CG_PQ3(false, false);
#undef PSW_CG_PQ3
    return e;
}

// r -= alpha q with alpha = rz / (sum of npq p.q partials); out[0] = p.q, out[1] = alpha,
// out[2 + b] = block b's partial of r.r (kRedBlocks of them).  The same values go to hout
// (pinned host memory, device-visible) when given, for the host's stopping test.
__global__ void __launch_bounds__(kRedThreads) k_cg_r(double *r, const double *q, const double *rz,
                                                     const double *pq_part, int npq, double *out, int64_t N,
                                                     double *hout) {
    __shared__ double sh[kRedThreads];
    const double pq = wave_sum_partials(pq_part, npq);
    const double alpha = rz[0] / pq;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        out[0] = pq;
        out[1] = alpha;
        if (hout) {
            hout[0] = pq;
            hout[1] = alpha;
        }
    }
    double acc = 0.0;
    const int64_t stride = (int64_t)kRedBlocks * kRedThreads;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < N; i += stride) {
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        acc += ri * ri;
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) {
        out[2 + blockIdx.x] = s;
        if (hout) hout[2 + blockIdx.x] = s;
    }
}

hipError_t launch_cg_r(double *r, const double *q, const double *rz, const double *pq_part, int npq, double *out,
                       int64_t N, double *hout, hipStream_t st) {
    hipLaunchKernelGGL(k_cg_r, dim3(kRedBlocks), dim3(kRedThreads), 0, st, r, q, rz, pq_part, npq, out, N, hout);
    return hipGetLastError();
}

__global__ void k_axpy_dev(double *y, const double *a, const double *x, int64_t N) {
    const double s = a[0];
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        y[i] += s * x[i];
}

hipError_t launch_axpy_dev(double *y, const double *a, const double *x, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_axpy_dev, dim3(grid_for(N)), dim3(256), 0, st, y, a, x, N);
    return hipGetLastError();
}

__global__ void k_copy_scaled(double *y, const double *x, double a, int64_t N) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a * x[i];
}

hipError_t launch_copy_scaled(double *y, const double *x, double a, int64_t N, hipStream_t st) {
    hipLaunchKernelGGL(k_copy_scaled, dim3(grid_for(N)), dim3(256), 0, st, y, x, a, N);
    return hipGetLastError();
}

__global__ void k_multi_axpy(double *y, const double *V, const double *c, int k, int64_t N, int accumulate) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x) {
        double acc = accumulate ? y[i] : 0.0;
        for (int j = 0; j < k; ++j) acc += c[j] * V[(int64_t)j * N + i];
        y[i] = acc;
    }
}

hipError_t launch_multi_axpy(double *y, const double *V, const double *c, int k, int64_t N, bool accumulate,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_multi_axpy, dim3(grid_for(N)), dim3(256), 0, st, y, V, c, k, N, accumulate ? 1 : 0);
    return hipGetLastError();
}

__global__ void __launch_bounds__(kRedThreads) k_multi_dot_partial(const double *V, const double *w, int64_t N,
                                                                  double *partials) {
    __shared__ double sh[kRedThreads];
    const int j = blockIdx.y;
    const double *v = V + (int64_t)j * N;
    double acc = 0.0;
    const int64_t stride = (int64_t)kRedBlocks * kRedThreads;
    for (int64_t i = blockIdx.x * (int64_t)kRedThreads + threadIdx.x; i < N; i += stride) acc += v[i] * w[i];
    double s = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[(int64_t)j * kRedBlocks + blockIdx.x] = s;
}

hipError_t launch_multi_dot(const double *V, const double *w, int k, int64_t N, double *partials, double *out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_multi_dot_partial, dim3(kRedBlocks, k), dim3(kRedThreads), 0, st, V, w, N, partials);
    hipLaunchKernelGGL(k_dot_final, dim3(k), dim3(kRedThreads), 0, st, partials, out);
    return hipGetLastError();
}


// ------------------------------------------------------------------ 3D half-sweeps with the tile in LDS
// For FP32 arithmetic (FP32 or BF16 storage) a whole 3D tile fits in LDS.  The
// workgroup stages the tile's input with row loads along x, sweeps it level by
// level (level t = l0 + l1 + l2 in local orientation, one barrier per level)
// with the results written in place, and writes the tile back with row stores.
// Thread c owns pencil c = l1 + L1 l2 and handles l0 = t - l1 - l2 at level t;
// its upstream neighbours sit at -1, -pitch and -pitch L1 in the pencil-major
// LDS tile.  Coefficients come packed per pass in level-major order, slot
// t C + c, so that one level's loads are contiguous: 1/Piv and the three
// upstream couplings divided by Piv, in the storage precision, read PD levels
// ahead.  Start-coupled passes solve the coupled blocks at the start faces
// (2x2 on faces, 4x4 on edges, 8x8 at the corner) as the generic kernel does,
// with the partners' values in LDS rings.
template <typename S> struct alignas(4 * sizeof(S)) Pk3 {
    S inv, c0, c1, c2;
};

__host__ __device__ __forceinline__ int tile3_pitch(int len0) { return len0 + (len0 & 1); } // pitch - 1 odd

size_t tile3_lds_bytes(const PassGeom &g, int len0max, size_t elem) {
    return elem * (size_t)tile3_pitch(len0max) * g.cmax;
}

__device__ __forceinline__ float s2f(float v) { return v; }
__device__ __forceinline__ float s2f(uint16_t v) { return bf16_to_f32(v); }
template <typename S> __device__ __forceinline__ S f2s(double v);
template <> __device__ __forceinline__ float f2s<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ uint16_t f2s<uint16_t>(double v) { return f64_to_bf16(v); }

// packed coefficients of one pass; transposed: couplings of the upstream
// neighbour towards the point (end-coupled passes), else of the point towards it
template <typename S>
__global__ void __launch_bounds__(256) k_pack3(PassGeom g, int transposed, DiagPtrs dg, const double *piv,
                                               const int64_t *poff, Pk3<S> *pk) {
    const TileDesc td = g.tiles[blockIdx.x];
    const TileFrame F = make_frame<3>(g, td);
    const int len0 = F.len[0], L1 = F.len[1], L2 = F.len[2], C = L1 * L2;
    Pk3<S> *out = pk + poff[blockIdx.x];
    for (int e = threadIdx.x; e < len0 * C; e += blockDim.x) {
        const int l0 = e % len0, c = e / len0;
        const int l[3] = {l0, c % L1, c / L1};
        int gp[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) gp[a] = F.base[a] + F.d[a] * l[a];
        const int64_t P = lin(g.n, gp);
        const double inv = 1.0 / piv[P];
        double cf[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            cf[a] = 0.0;
            if (l[a] > 0) {
                if (transposed) {
                    int r[3] = {gp[0], gp[1], gp[2]};
                    r[a] -= F.d[a];
                    cf[a] = dg.d[dk(a, F.d[a])][lin(g.n, r)] * inv;
                } else {
                    cf[a] = dg.d[dk(a, -F.d[a])][P] * inv;
                }
            }
        }
        Pk3<S> v;
        v.inv = f2s<S>(inv);
        v.c0 = f2s<S>(cf[0]);
        v.c1 = f2s<S>(cf[1]);
        v.c2 = f2s<S>(cf[2]);
        out[(int64_t)(l[0] + l[1] + l[2]) * C + c] = v;
    }
}

template <typename S, typename TIN, typename TOUT> struct Tile3Args {
    PassGeom g;
    const S *diag[7];
    const S *piv;
    const Pk3<S> *pk;
    const int64_t *poff;
    const TIN *in;
    int scale_by_piv;
    TOUT *out;
    double cscale;
    int len0max;
};

constexpr int kTile3Pd = 8; // levels by which the packed coefficients are read ahead

template <typename T, typename S, typename TIN, typename TOUT, bool CPL>
__global__ void __launch_bounds__(1024) k_tile3(Tile3Args<S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PassGeom &g = A.g;
    const TileDesc td = g.tiles[blockIdx.x];
    const TileFrame F = make_frame<3>(g, td);
    const int len0 = F.len[0], L1 = F.len[1], L2 = F.len[2];
    const int C = L1 * L2;
    const int nlev = len0 + L1 + L2 - 2;
    const int pitch = tile3_pitch(len0);
    T *own = reinterpret_cast<T *>(smem);
    const int nth = blockDim.x;
    const int np = len0 * C;
    // the input, and for a start-coupled pass the values of the coupled start-face points,
    // which the level kernel has already solved into out (unscaled).  Row-wise: thread t takes
    // column x = t % XS of the rows (pencils) t / XS + k RPI, U rows at a time with all their
    // loads in flight before the LDS stores.  The loads are unconditional (a guarded load gets
    // its conversion, and so a wait, inside the guard; a row past the tile reads its first row),
    // and the coordinates and addresses advance by fixed steps (the index arithmetic of a general
    // element order costs more than the copy).
    auto on_face = [&](int l0, int l1, int l2) {
        return CPL && ((l0 == 0 && F.start_cpl[0]) || (l1 == 0 && F.start_cpl[1]) || (l2 == 0 && F.start_cpl[2]));
    };
    const int XS = min(len0, nth), RPI = max(1, nth / len0);
    const int tx = threadIdx.x % XS, tc = threadIdx.x / XS;
    const int64_t gs0 = F.d[0], gs1 = (int64_t)F.d[1] * g.n[0], gs2 = (int64_t)F.d[2] * g.n[0] * g.n[1];
    const int64_t gb = lin(g.n, F.base);
    const int dl1 = RPI % L1, dl2 = RPI / L1;
    const int64_t dg = dl1 * gs1 + dl2 * gs2, wrapg = gs2 - (int64_t)L1 * gs1;
    // row c -> (l1, l2) and its global index at column x
    auto row_at = [&](int c, int x, int &l1, int &l2, int64_t &gi) {
        l1 = c % L1;
        l2 = c / L1;
        gi = gb + x * gs0 + l1 * gs1 + l2 * gs2;
    };
    auto advance = [&](int &l1, int &l2, int64_t &gi) {
        l1 += dl1;
        l2 += dl2;
        gi += dg;
        if (l1 >= L1) {
            l1 -= L1;
            ++l2;
            gi += wrapg;
        }
    };
    constexpr int U = 16;
    if (tc < RPI) {
        for (int x = tx; x < len0; x += XS) {
            const int64_t gx = gb + x * gs0;
            for (int c0 = tc; c0 < C; c0 += U * RPI) {
                int l1, l2;
                int64_t gi;
                row_at(c0, x, l1, l2, gi);
                TIN v[U];
                unsigned keep = 0;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool in = c0 + u * RPI < C;
                    v[u] = __builtin_nontemporal_load(&A.in[in ? gi : gx]); // read once: streaming load
                    if (in && !on_face(x, l1, l2)) keep |= 1u << u;
                    advance(l1, l2, gi);
                }
#pragma unroll
                for (int u = 0; u < U; ++u)
                    if ((keep >> u) & 1u) own[(c0 + u * RPI) * pitch + x] = cvt_in<T>(v[u]);
            }
        }
    }
    if (CPL) {
        // the coupled start-face points: a point on two faces is written twice with one value
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            if (!F.start_cpl[a]) continue;
            const int lb = a == 0 ? L1 : len0, nf = a == 2 ? len0 * L1 : (a == 1 ? len0 * L2 : L1 * L2);
            for (int j = threadIdx.x; j < nf; j += nth) {
                const int u = j % lb, w = j / lb;
                const int l0 = a == 0 ? 0 : u, l1 = a == 1 ? 0 : (a == 0 ? u : w), l2 = a == 2 ? 0 : w;
                const int gp[3] = {F.base[0] + F.d[0] * l0, F.base[1] + F.d[1] * l1, F.base[2] + F.d[2] * l2};
                own[(l1 + L1 * l2) * pitch + l0] = ldv<T>((const TOUT *)A.out, lin(g.n, gp));
            }
        }
    }
    __syncthreads();

    const int c = threadIdx.x;
    const bool have = c < C;
    const int l1 = have ? c % L1 : 0, l2 = have ? c / L1 : 0;
    const Pk3<S> *pk = A.pk + A.poff[blockIdx.x] + (have ? c : 0); // threads beyond the tile read slot 0
    const bool scale = A.scale_by_piv != 0;
    constexpr int PD = kTile3Pd;
    // The ring's loads are issued by every lane at every level, and each slot is reloaded after
    // its last use in the level, so the slot keeps its registers and no wait is needed before the
    // level's barrier.  The ring is filled in level order (a scheduling barrier after each load
    // keeps the compiler from issuing them in another order): the wait before level t's
    // coefficients is then for the load issued PD levels earlier, with the younger loads still in
    // flight.  A load under a branch (or issued in reverse order) makes every level wait for all
    // outstanding loads.  A pencil with no point at a level reads the tile's first slot instead
    // of its own: the level-major layout keeps a slot for every (level, pencil) pair, about
    // (len0 + L1 + L2 - 2) / len0 times the point count, and reading them all would move that
    // many times the coefficient bytes, while the one shared slot stays in cache.
    const Pk3<S> *pk0 = A.pk + A.poff[blockIdx.x];
    const int o = l1 + l2;
    auto slot = [&](int t) -> const Pk3<S> * {
        return (have && (unsigned)(t - o) < (unsigned)len0) ? pk + (int64_t)t * C : pk0;
    };
    Pk3<S> ring[PD];
#pragma unroll
    for (int k = 0; k < PD; ++k) {
        ring[k] = *slot(k);
        __builtin_amdgcn_sched_barrier(0);
    }
    // whole blocks of PD levels: the levels past the last one hold no point (no branch around
    // the ring's loads)
    for (int t0 = 0; t0 < nlev; t0 += PD) {
#pragma unroll
        for (int k = 0; k < PD; ++k) {
            const int t = t0 + k;
            {
                const Pk3<S> &cf = ring[k];
                const int l0 = t - l1 - l2;
                if (have && l0 >= 0 && l0 < len0) {
                    int Am = 0;
                    if (CPL) {
                        if (l0 == 0 && F.start_cpl[0]) Am |= 1;
                        if (l1 == 0 && F.start_cpl[1]) Am |= 2;
                        if (l2 == 0 && F.start_cpl[2]) Am |= 4;
                    }
                    const int o = c * pitch + l0;
                    if (Am == 0) {
                        // the four reads issued together: a missing upstream neighbour (l = 0) has a
                        // packed weight of exactly zero and reads the point itself (finite)
                        const int o0 = l0 > 0 ? o - 1 : o, o1 = l1 > 0 ? o - pitch : o, o2 = l2 > 0 ? o - pitch * L1 : o;
                        T acc = own[o];
                        const T u0 = own[o0], u1 = own[o1], u2 = own[o2];
                        if (!scale) acc *= s2f(cf.inv);
                        acc = __fmaf_rn(s2f(cf.c0), u0, acc);
                        acc = __fmaf_rn(s2f(cf.c1), u1, acc);
                        acc = __fmaf_rn(s2f(cf.c2), u2, acc);
                        own[o] = acc;
                    }
                }
                ring[k] = *slot(t + PD);
                lds_barrier();
            }
        }
    }
    // write-back with streaming stores: the output lines are not read again by this pass
    const T cs = (T)A.cscale;
    if (tc < RPI) {
        for (int x = tx; x < len0; x += XS) {
            for (int c0 = tc; c0 < C; c0 += U * RPI) {
                int l1w, l2w;
                int64_t gi;
                row_at(c0, x, l1w, l2w, gi);
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int cr = c0 + u * RPI;
                    if (cr < C) __builtin_nontemporal_store((TOUT)(cs * own[cr * pitch + x]), &A.out[gi]);
                    advance(l1w, l2w, gi);
                }
            }
        }
    }
}

hipError_t launch_pack3(const PassGeom &g, Store s, bool transposed, const double *const *diag, const double *piv,
                        const int64_t *poff, void *pk, hipStream_t st) {
    if (g.dim != 3 || s == Store::F64) return hipErrorInvalidValue;
    DiagPtrs D{};
    for (int k = 0; k < 7; ++k) D.d[k] = diag[k];
    if (s == Store::F32)
        hipLaunchKernelGGL(k_pack3<float>, dim3(g.ntiles), dim3(256), 0, st, g, (int)transposed, D, piv, poff,
                           (Pk3<float> *)pk);
    else
        hipLaunchKernelGGL(k_pack3<uint16_t>, dim3(g.ntiles), dim3(256), 0, st, g, (int)transposed, D, piv, poff,
                           (Pk3<uint16_t> *)pk);
    return hipGetLastError();
}

size_t pack3_slot_bytes(Store s) { return s == Store::F32 ? sizeof(Pk3<float>) : sizeof(Pk3<uint16_t>); }

template <typename S, typename TIN, typename TOUT>
static hipError_t tile3_impl(const PassGeom &g, bool start, const void *const *diag, const void *piv, const void *pk,
                             const int64_t *poff, int len0max, const void *in, bool scale_by_piv, void *out,
                             double cscale, void *fimg, hipStream_t st) {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds = 0;
    Tile3Args<S, TIN, TOUT> A{};
    A.g = g;
    for (int k = 0; k < 7; ++k) A.diag[k] = (const S *)diag[k];
    A.piv = (const S *)piv;
    A.pk = (const Pk3<S> *)pk;
    A.poff = poff;
    A.in = (const TIN *)in;
    A.scale_by_piv = scale_by_piv ? 1 : 0;
    A.out = (TOUT *)out;
    A.cscale = cscale;
    A.len0max = len0max;
    if (g.cmax > 1024) return hipErrorInvalidValue;
    const int nth = std::max(64, (g.cmax + 63) / 64 * 64);
    const size_t sm = tile3_lds_bytes(g, len0max, sizeof(float));
    if (start) {
        // the coupled start faces first (level kernel, faces only, unscaled into out)
        hipError_t e =
            start_impl<float, S, TIN, TOUT>(g, diag, piv, in, scale_by_piv, out, 1.0, st, true, len0max, (size_t)lds,
                                            fimg, 2);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_tile3<float, S, TIN, TOUT, true>), dim3(g.ntiles), dim3(nth), sm, st, A);
    }
    else
        hipLaunchKernelGGL((k_tile3<float, S, TIN, TOUT, false>), dim3(g.ntiles), dim3(nth), sm, st, A);
    return hipGetLastError();
}

hipError_t launch_tile3(const PassGeom &g, Store s, bool start, const void *const *diag, const void *piv,
                        const void *pk, const int64_t *poff, int len0max, const void *in, bool in_f64,
                        bool scale_by_piv, void *out, bool out_f64, double cscale, void *fimg, hipStream_t st) {
    if (g.dim != 3 || s == Store::F64) return hipErrorInvalidValue;
#define PSW_T3(S, TIN, TOUT) \
    tile3_impl<S, TIN, TOUT>(g, start, diag, piv, pk, poff, len0max, in, scale_by_piv, out, cscale, fimg, st)
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return PSW_T3(float, double, float);
        if (!in_f64 && out_f64) return PSW_T3(float, float, double);
        if (in_f64 && out_f64) return PSW_T3(float, double, double);
        return PSW_T3(float, float, float);
    }
    if (in_f64 && !out_f64) return PSW_T3(uint16_t, double, float);
    if (!in_f64 && out_f64) return PSW_T3(uint16_t, float, double);
    if (in_f64 && out_f64) return PSW_T3(uint16_t, double, double);
    return PSW_T3(uint16_t, float, float);
#undef PSW_T3
}

// Elements of the coefficient image of a start-coupled 3D pass (all tiles), 0 if the
// gathered-record face kernel does not apply to these tiles.
int64_t faces3_image_elems(const PassGeom &g, int len0max, size_t lds_limit) {
    if (g.dim != 3 || g.cmax > 1024 || len0max <= 0) return 0;
    const int lmax = std::max(len0max, std::max(g.l1max, g.l2max));
    const int fmax = faces3_rec_floats(len0max, g.l1max, g.l2max, lmax);
    if (faces3_lds_bytes(g, fmax, sizeof(float)) > lds_limit) return 0;
    return (int64_t)fmax * g.ntiles;
}

// Write the coefficient image of a start-coupled 3D pass: per tile, the records of its
// coupled start faces with the pivot where the right-hand side goes (FP32 sweeps).
hipError_t launch_faces3_image(const PassGeom &g, Store s, const void *const *diag, const void *piv, int len0max,
                               size_t lds_limit, void *img, hipStream_t st) {
    if (g.dim != 3 || s == Store::F64 || !img) return hipErrorInvalidValue;
    if (s == Store::F32)
        return start_impl<float, float, double, double>(g, diag, piv, nullptr, false, nullptr, 1.0, st, true, len0max,
                                                        lds_limit, img, 1);
    return start_impl<float, uint16_t, double, double>(g, diag, piv, nullptr, false, nullptr, 1.0, st, true, len0max,
                                                       lds_limit, img, 1);
}

// the coupled end faces, edges and corners of an end-coupled 3D pass (after its interior)
hipError_t launch_end_fixups3(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                              bool in_f64, bool scale_by_piv, void *out, bool out_f64, int len0max, void *eimg,
                              hipStream_t st) {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        lds = 0;
    return end_part(g, s, diag, piv, in, in_f64, scale_by_piv, out, out_f64, 2, st, len0max, (size_t)lds, eimg,
                    eimg ? 2 : 0);
}

int64_t end_faces3_image_elems(const PassGeom &g, int len0max, size_t lds_limit) {
    if (g.dim != 3 || len0max <= 0) return 0;
    const int fmax = std::max(g.l1max * g.l2max, len0max * std::max(g.l1max, g.l2max));
    if (fmax > 1024 || kEndImg * (size_t)fmax * sizeof(float) > lds_limit) return 0;
    return kEndImg * (int64_t)fmax * g.ntiles * 3;
}

hipError_t launch_end_faces3_image(const PassGeom &g, Store s, const void *const *diag, const void *piv, int len0max,
                                   size_t lds_limit, void *img, hipStream_t st) {
    if (g.dim != 3 || s == Store::F64 || !img) return hipErrorInvalidValue;
    return end_part(g, s, diag, piv, nullptr, true, false, nullptr, true, 2, st, len0max, lds_limit, img, 1);
}

} // namespace psw
