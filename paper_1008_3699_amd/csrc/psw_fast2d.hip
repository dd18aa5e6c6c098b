// psw_fast2d.hip -- wavefront-pipelined 2D half-sweep kernels for gfx950.
//
// One workgroup per tile.  The tile is swept in its local orientation
// (towards +x, +y).  One 64-lane wave carries the recurrence: lane j owns R
// consecutive rows and handles column x = s - j at step s, so each step is a
// whole anti-diagonal of the tile (the frontal sweep of Sec. 2) and lane j
// receives the new value of the row above it from lane j-1 by a cross-lane
// shuffle.  The input vector tile (plus the partner column / row across the
// coupled start faces) is staged in LDS by the whole workgroup with
// coalesced row loads; the results go back through LDS the same way.
//
// The per-point coefficients of a pass (1/Piv and the two upstream couplings
// multiplied by 1/Piv) are packed once per problem in "sweep-major" order:
// step s, lane j, row r at ((s*64 + j)*R + r), so that each step of the
// wave reads one contiguous 64*R-element burst per array.  The wave keeps a
// ring of kDepth steps of these loads in flight.
//
// Start-coupled passes solve the coupled blocks at the tile's start faces
// inside the pipeline (2x2 pairs chained along each face, 4x4 at the cross
// point; eq. 2d:sor2b2 / eq. 2d:sor4b4 with Piv in place of a^P/omega).
#include "psw_internal.h"
#include "psw_fast2d.h"

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psw {

namespace {

__device__ __forceinline__ float bf16f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

__device__ __forceinline__ uint16_t to_bf16(double x) {
    float t = __double2float_rz(x);
    uint32_t u = __float_as_uint(t);
    if ((double)t != x && (u & 0x7f800000u) != 0x7f800000u) u |= 1u;
    uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}

template <typename S> __device__ __forceinline__ S from_f64(double v);
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f64<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ uint16_t from_f64<uint16_t>(double v) { return to_bf16(v); }

template <typename T, typename S> __device__ __forceinline__ T cvt(S v);
template <> __device__ __forceinline__ double cvt<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt<float, float>(float v) { return v; }
template <> __device__ __forceinline__ float cvt<float, double>(double v) { return (float)v; }
template <> __device__ __forceinline__ double cvt<double, float>(float v) { return (double)v; }
template <> __device__ __forceinline__ float cvt<float, uint16_t>(uint16_t v) { return bf16f(v); }

__device__ __forceinline__ int dkk(int a, int s) { return s < 0 ? 1 + 2 * a : 2 + 2 * a; }

__device__ __forceinline__ int64_t lin2(int n0, int gx, int gy) { return (int64_t)gx + (int64_t)n0 * gy; }

// R values of storage type S for one lane and step, loaded as one vector
template <typename S, int R> struct Pack;
template <> struct Pack<double, 1> { using V = double; };
template <> struct Pack<double, 2> { using V = double2; };
template <> struct Pack<float, 1> { using V = float; };
template <> struct Pack<float, 2> { using V = float2; };
template <> struct Pack<uint16_t, 1> { using V = uint16_t; };
template <> struct Pack<uint16_t, 2> { using V = uint32_t; };

template <typename T, typename V> __device__ __forceinline__ T elem(const V &v, int r);
template <> __device__ __forceinline__ double elem<double, double>(const double &v, int) { return v; }
template <> __device__ __forceinline__ double elem<double, double2>(const double2 &v, int r) { return r ? v.y : v.x; }
template <> __device__ __forceinline__ float elem<float, float>(const float &v, int) { return v; }
template <> __device__ __forceinline__ float elem<float, float2>(const float2 &v, int r) { return r ? v.y : v.x; }
template <> __device__ __forceinline__ float elem<float, uint16_t>(const uint16_t &v, int) { return bf16f(v); }
template <> __device__ __forceinline__ float elem<float, uint32_t>(const uint32_t &v, int r) {
    return __uint_as_float(r ? (v & 0xffff0000u) : (v << 16));
}

struct Frame2 {
    int d0, d1, lx, ly, lox, loy;
    bool cx, cy; // coupled start faces
};

__device__ __forceinline__ Frame2 frame2(const PassGeom &g, const TileDesc &td) {
    Frame2 f;
    f.d0 = g.sig[0] * (td.par[0] ? -1 : 1);
    f.d1 = g.sig[1] * (td.par[1] ? -1 : 1);
    f.lx = td.len[0];
    f.ly = td.len[1];
    f.lox = td.lo[0];
    f.loy = td.lo[1];
    f.cx = f.d0 > 0 ? td.lo[0] > 0 : td.lo[0] + td.len[0] < g.n[0];
    f.cy = f.d1 > 0 ? td.lo[1] > 0 : td.lo[1] + td.len[1] < g.n[1];
    return f;
}

// global coordinate of local coordinate l (l = -1 is the partner across the start face)
__device__ __forceinline__ int gx_of(const Frame2 &f, int x) { return f.d0 > 0 ? f.lox + x : f.lox + f.lx - 1 - x; }
__device__ __forceinline__ int gy_of(const Frame2 &f, int y) { return f.d1 > 0 ? f.loy + y : f.loy + f.ly - 1 - y; }

} // namespace

// ------------------------------------------------------------------ packing
// Coefficients of one pass in sweep-major order plus the partner data of the
// coupled start faces.  transposed: the couplings are those of the upstream
// neighbour towards the point (a_{R->P}) and no face is coupled.
template <typename S>
__global__ void k_pack2d(PassGeom g, int R, int transposed, Fast2dDiag dg, const double *__restrict__ piv,
                         const int64_t *__restrict__ toff, const int64_t *__restrict__ foff, S *s_inv, S *s_ax,
                         S *s_ay, S *face) {
    const TileDesc td = g.tiles[blockIdx.x];
    const Frame2 F = frame2(g, td);
    const bool cx = !transposed && F.cx, cy = !transposed && F.cy;
    const int L = (F.ly + R - 1) / R;
    const int64_t nslots = (int64_t)(F.lx + L - 1 + kFast2dDepth) * 64 * R;
    const int64_t base = toff[blockIdx.x];
    const int n0 = g.n[0];
    for (int64_t sl = threadIdx.x; sl < nslots; sl += blockDim.x) {
        const int r = (int)(sl % R), j = (int)((sl / R) % 64);
        const int s = (int)(sl / (64 * R));
        const int x = s - j, y = R * j + r;
        double inv = 0, ax = 0, ay = 0;
        if (j < L && x >= 0 && x < F.lx && y < F.ly) {
            const int gx = gx_of(F, x), gy = gy_of(F, y);
            const int64_t P = lin2(n0, gx, gy);
            inv = 1.0 / piv[P];
            if (x > 0 || cx) {
                const int64_t Q = lin2(n0, gx - F.d0, gy);
                ax = (transposed ? dg.d[dkk(0, +F.d0)][Q] : dg.d[dkk(0, -F.d0)][P]) * inv;
            }
            if (y > 0 || cy) {
                const int64_t Q = lin2(n0, gx, gy - F.d1);
                ay = (transposed ? dg.d[dkk(1, +F.d1)][Q] : dg.d[dkk(1, -F.d1)][P]) * inv;
            }
        }
        s_inv[base + sl] = from_f64<S>(inv);
        s_ax[base + sl] = from_f64<S>(ax);
        s_ay[base + sl] = from_f64<S>(ay);
    }
    // partner data of the coupled start faces: [inv, a'_{Q->P}, a'_{Q->upstream}] per row / column
    S *fc = face + foff[blockIdx.x];
    for (int y = threadIdx.x; y < F.ly; y += blockDim.x) {
        double v0 = 0, v1 = 0, v2 = 0;
        if (cx) {
            const int gx = gx_of(F, -1), gy = gy_of(F, y);
            const int64_t Q = lin2(n0, gx, gy);
            v0 = 1.0 / piv[Q];
            v1 = dg.d[dkk(0, +F.d0)][Q] * v0;
            if (y > 0 || cy) v2 = dg.d[dkk(1, -F.d1)][Q] * v0;
        }
        fc[y] = from_f64<S>(v0);
        fc[F.ly + y] = from_f64<S>(v1);
        fc[2 * F.ly + y] = from_f64<S>(v2);
    }
    S *fr = fc + 3 * F.ly;
    for (int x = threadIdx.x; x < F.lx; x += blockDim.x) {
        double v0 = 0, v1 = 0, v2 = 0;
        if (cy) {
            const int gx = gx_of(F, x), gy = gy_of(F, -1);
            const int64_t Q = lin2(n0, gx, gy);
            v0 = 1.0 / piv[Q];
            v1 = dg.d[dkk(1, +F.d1)][Q] * v0;
            if (x > 0 || cx) v2 = dg.d[dkk(0, -F.d0)][Q] * v0;
        }
        fr[x] = from_f64<S>(v0);
        fr[F.lx + x] = from_f64<S>(v1);
        fr[2 * F.lx + x] = from_f64<S>(v2);
    }
    if (threadIdx.x == 0) {
        S *fk = fr + 3 * F.lx;
        double v0 = 0, v1 = 0, v2 = 0;
        if (cx && cy) {
            const int64_t Q = lin2(n0, gx_of(F, -1), gy_of(F, -1));
            v0 = 1.0 / piv[Q];
            v1 = dg.d[dkk(1, +F.d1)][Q] * v0; // towards (-1, 0)
            v2 = dg.d[dkk(0, +F.d0)][Q] * v0; // towards (0, -1)
        }
        fk[0] = from_f64<S>(v0);
        fk[1] = from_f64<S>(v1);
        fk[2] = from_f64<S>(v2);
    }
}

// ------------------------------------------------------------------ the pipelined half-sweep
template <typename S, typename TIN, typename TOUT> struct Fast2dArgs {
    PassGeom g;
    const S *s_inv, *s_ax, *s_ay, *face;
    const int64_t *toff, *foff;
    const TIN *in;
    TOUT *out;
    int scale_by_piv; // rhs' = in (backward passes) instead of in / Piv
    int coupled;      // start faces coupled (0 for the transposed passes)
    double cscale;
    int pitch_max;
};

template <typename T> __device__ __forceinline__ T shfl_up1(T v) { return __shfl_up(v, 1, 64); }

template <int R, typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(256) k_fast2d(Fast2dArgs<S, TIN, TOUT> A) {
    using V = typename Pack<S, R>::V;
    constexpr int D = kFast2dDepth;
    extern __shared__ __align__(16) unsigned char smem[];
    const PassGeom &g = A.g;
    const TileDesc td = g.tiles[blockIdx.x];
    const Frame2 F = frame2(g, td);
    const bool cx = A.coupled && F.cx, cy = A.coupled && F.cy;
    const int lx = F.lx, ly = F.ly;
    // LDS: vector tile in global orientation with a one-point ring, pitch chosen
    // so that the wave's anti-diagonal reads hit distinct banks
    int pitch = lx + 2;
    if ((R * pitch) & 1) ++pitch;
    T *vt = reinterpret_cast<T *>(smem);
    T *fx = vt + (size_t)(ly + 2) * pitch; // x-face partners: inv, a'QP, a'Qy (ly each)
    T *fy = fx + 3 * ly;                   // y-face partners (lx each)
    T *fk = fy + 3 * lx;                   // cross point partner
    const int n0 = g.n[0];
    const int tid = threadIdx.x, nth = blockDim.x;

    // ---- stage the input tile (+ partners) into LDS, coalesced along rows
    for (int idx = tid; idx < lx * ly; idx += nth) {
        const int row = idx / lx, col = idx - row * lx;
        const int gx = F.lox + col, gy = F.loy + row;
        vt[(row + 1) * pitch + col + 1] = cvt<T>(A.in[lin2(n0, gx, gy)]);
    }
    if (cx) {
        const int gx = gx_of(F, -1), col = F.d0 > 0 ? 0 : lx + 1;
        for (int row = tid; row < ly; row += nth) vt[(row + 1) * pitch + col] = cvt<T>(A.in[lin2(n0, gx, F.loy + row)]);
    }
    if (cy) {
        const int gy = gy_of(F, -1), row = F.d1 > 0 ? 0 : ly + 1;
        for (int col = tid; col < lx; col += nth) vt[row * pitch + col + 1] = cvt<T>(A.in[lin2(n0, F.lox + col, gy)]);
    }
    if (cx && cy && tid == 0) {
        const int col = F.d0 > 0 ? 0 : lx + 1, row = F.d1 > 0 ? 0 : ly + 1;
        vt[row * pitch + col] = cvt<T>(A.in[lin2(n0, gx_of(F, -1), gy_of(F, -1))]);
    }
    const S *fsrc = A.face + A.foff[blockIdx.x];
    for (int i = tid; i < 3 * (lx + ly) + 3; i += nth) fx[i] = cvt<T>(fsrc[i]);
    __syncthreads();

    // ---- the recurrence: wave 0
    if (tid < 64) {
        const int lane = tid;
        const int L = (ly + R - 1) / R;
        const int nr = lane < L ? min(R, ly - R * lane) : 0;
        const int nsteps = lx + L - 1;
        const int64_t sbase = A.toff[blockIdx.x];
        const V *pinv = reinterpret_cast<const V *>(A.s_inv + sbase);
        const V *pax = reinterpret_cast<const V *>(A.s_ax + sbase);
        const V *pay = reinterpret_cast<const V *>(A.s_ay + sbase);
        const bool sc = A.scale_by_piv != 0;
        // LDS addressing in local orientation
        const int cstep = F.d0 > 0 ? 1 : -1, col0 = F.d0 > 0 ? 1 : lx; // column of local x = 0
        const int rstep = F.d1 > 0 ? pitch : -pitch, row0 = (F.d1 > 0 ? 1 : ly) * pitch;
        const int rowbase = row0 + rstep * (R * lane);
        V ri[D], ra[D], rb[D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int x = k - lane;
            const bool act = nr > 0 && x >= 0 && x < lx;
            if (act) {
                const int64_t o = (int64_t)k * 64 + lane;
                if (!sc) ri[k] = pinv[o];
                ra[k] = pax[o];
                rb[k] = pay[o];
            }
        }
        T left[R];
#pragma unroll
        for (int r = 0; r < R; ++r) left[r] = T(0);
        T last = T(0);    // value of this lane's last row at the previous step
        T xplast = T(0);  // x-face partner of this lane's last row (set at x = 0)
        T yprev = T(0);   // y-face partner at the previous column (lane 0)
        for (int s0 = 0; s0 < nsteps; s0 += D) {
#pragma unroll
            for (int k = 0; k < D; ++k) {
                const int s = s0 + k;
                if (s < nsteps) {
                    const T up_in = shfl_up1(last);
                    const T upx_in = shfl_up1(xplast);
                    const int x = s - lane;
                    if (nr > 0 && x >= 0 && x < lx) {
                        T up = (lane > 0) ? up_in : T(0);
                        T upx = (lane > 0) ? upx_in : T(0);
                        const int cidx = col0 + cstep * x;
                        T v = T(0), vq = T(0);
#pragma unroll
                        for (int r = 0; r < R; ++r) {
                            if (r < nr) {
                                const int y = R * lane + r;
                                const int a = rowbase + rstep * r + cidx;
                                const T iv = sc ? T(1) : elem<T>(ri[k], r);
                                const T ax = elem<T>(ra[k], r), ay = elem<T>(rb[k], r);
                                const T rhs = sc ? vt[a] : iv * vt[a];
                                if (x == 0 && cx) {
                                    // x-face partner Q = (-1, y)
                                    const int aq = a - cstep;
                                    const T ivq = fx[y], aqp = fx[ly + y], aqy = fx[2 * ly + y];
                                    const T rq = sc ? vt[aq] : ivq * vt[aq];
                                    if (y == 0 && cy) {
                                        // cross point: A=(0,0), B=(-1,0), C=(0,-1), D=(-1,-1)
                                        const T ivc = fy[0], acp = fy[lx], acd = fy[2 * lx];
                                        const T ivd = fk[0], adb = fk[1], adc = fk[2];
                                        const int ac = a - rstep, ad = a - rstep - cstep;
                                        const T rc = sc ? vt[ac] : ivc * vt[ac];
                                        const T rd = sc ? vt[ad] : ivd * vt[ad];
                                        // rows: A: yA - ax yB - ay yC = rhs ; B: yB - aqp yA - aqy yD = rq
                                        //       C: yC - acp yA - acd yD = rc ; D: yD - adb yB - adc yC = rd
                                        T M[4][4] = {{T(1), -ax, -ay, T(0)},
                                                     {-aqp, T(1), T(0), -aqy},
                                                     {-acp, T(0), T(1), -acd},
                                                     {T(0), -adb, -adc, T(1)}};
                                        T b[4] = {rhs, rq, rc, rd};
#pragma unroll
                                        for (int p = 0; p < 4; ++p) {
                                            const T ip = T(1) / M[p][p];
#pragma unroll
                                            for (int i = p + 1; i < 4; ++i) {
                                                const T l = M[i][p] * ip;
#pragma unroll
                                                for (int jj = p + 1; jj < 4; ++jj) M[i][jj] -= l * M[p][jj];
                                                b[i] -= l * b[p];
                                            }
                                        }
#pragma unroll
                                        for (int i = 3; i >= 0; --i) {
                                            T acc = b[i];
#pragma unroll
                                            for (int jj = i + 1; jj < 4; ++jj) acc -= M[i][jj] * b[jj];
                                            b[i] = acc / M[i][i];
                                        }
                                        v = b[0];
                                        vq = b[1];
                                        yprev = b[2];
                                    } else {
                                        const T bp = rhs + ay * up;
                                        const T bq = rq + aqy * upx;
                                        const T det = T(1) - ax * aqp;
                                        v = (bp + ax * bq) / det;
                                        vq = (bq + aqp * bp) / det;
                                    }
                                } else if (y == 0 && cy) {
                                    // y-face partner Q = (x, -1), chained along x
                                    const int aq = a - rstep;
                                    const T ivq = fy[x], aqp = fy[lx + x], aqx = fy[2 * lx + x];
                                    const T rq = sc ? vt[aq] : ivq * vt[aq];
                                    const T bp = rhs + ax * left[r];
                                    const T bq = rq + aqx * yprev;
                                    const T det = T(1) - ay * aqp;
                                    v = (bp + ay * bq) / det;
                                    vq = (bq + aqp * bp) / det;
                                    yprev = vq;
                                } else {
                                    v = rhs + ax * left[r] + ay * up;
                                }
                                vt[a] = v;
                                left[r] = v;
                                up = v;
                                upx = vq;
                            }
                        }
                        last = up;
                        if (x == 0) xplast = upx;
                    }
                    // refill this ring slot with step s + D
                    const int xn = s + D - lane;
                    if (nr > 0 && xn >= 0 && xn < lx) {
                        const int64_t o = (int64_t)(s + D) * 64 + lane;
                        if (!sc) ri[k] = pinv[o];
                        ra[k] = pax[o];
                        rb[k] = pay[o];
                    }
                }
            }
        }
    }
    __syncthreads();

    // ---- write the tile back, coalesced along rows
    const T cs = (T)A.cscale;
    for (int idx = tid; idx < lx * ly; idx += nth) {
        const int row = idx / lx, col = idx - row * lx;
        A.out[lin2(n0, F.lox + col, F.loy + row)] = (TOUT)(cs * vt[(row + 1) * pitch + col + 1]);
    }
}

// ------------------------------------------------------------------ end-face chains (2D), prefetched
// The coupled end face owned by a tile (see k_end_faces in psw_kernels.hip):
// all data of the chain that does not depend on the chain itself is gathered
// into LDS by the workgroup; one thread then runs the 2x2 recurrence.
template <typename T, typename S, typename TIN, typename TOUT> struct EndFaceArgs {
    PassGeom g;
    const S *diag[5];
    const S *piv;
    const TIN *in;
    int scale_by_piv;
    TOUT *out;
};

template <typename T, typename S> __device__ __forceinline__ T ldS(const S *p, int64_t i) { return cvt<T>(p[i]); }

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(256) k_end_faces2d_fast(EndFaceArgs<T, S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const PassGeom &g = A.g;
    const int tile = blockIdx.x >> 1, a = blockIdx.x & 1, b = 1 - a;
    const TileDesc td = g.tiles[tile];
    int d[2], len[2], lo[2];
    bool endc[2];
    for (int q = 0; q < 2; ++q) {
        d[q] = g.sig[q] * (td.par[q] ? -1 : 1);
        len[q] = td.len[q];
        lo[q] = td.lo[q];
        endc[q] = d[q] > 0 ? lo[q] + len[q] < g.n[q] : lo[q] > 0;
    }
    if (!(d[a] > 0 && endc[a])) return;
    const int nb = endc[b] ? len[b] - 1 : len[b];
    T *mPQ = reinterpret_cast<T *>(smem);
    T *mQP = mPQ + nb, *cP = mQP + nb, *cQ = cP + nb, *bP = cQ + nb, *bQ = bP + nb;
    const int n0 = g.n[0];
    auto gidx = [&](int la, int lb) -> int64_t {
        int c[2];
        c[a] = d[a] > 0 ? lo[a] + la : lo[a] + len[a] - 1 - la;
        c[b] = d[b] > 0 ? lo[b] + lb : lo[b] + len[b] - 1 - lb;
        return (int64_t)c[0] + (int64_t)n0 * c[1];
    };
    // P at local (la = len_a-1, lb), Q at la = len_a (across), inward neighbours at len_a-2 and len_a+1
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        const int64_t P = gidx(len[a] - 1, k), Q = gidx(len[a], k);
        const int64_t Pin = gidx(len[a] - 2, k), Qin = gidx(len[a] + 1, k);
        const T DP = ldS<T>(A.piv, P), DQ = ldS<T>(A.piv, Q);
        T rp = cvt<T>(A.in[P]), rq = cvt<T>(A.in[Q]);
        if (A.scale_by_piv) {
            rp *= DP;
            rq *= DQ;
        }
        // couplings of the neighbours towards P / Q (transposed rows)
        const int sa = d[a], sb = d[b];
        rp += ldS<T>(A.diag[dkk(a, +sa)], Pin) * cvt<T>(A.out[Pin]);
        rq += ldS<T>(A.diag[dkk(a, -sa)], Qin) * cvt<T>(A.out[Qin]);
        mPQ[k] = ldS<T>(A.diag[dkk(a, -sa)], Q) / DP; // Q's coupling towards P
        mQP[k] = ldS<T>(A.diag[dkk(a, +sa)], P) / DQ; // P's coupling towards Q
        if (k > 0) {
            const int64_t Pp = gidx(len[a] - 1, k - 1), Qp = gidx(len[a], k - 1);
            cP[k] = ldS<T>(A.diag[dkk(b, +sb)], Pp) / DP;
            cQ[k] = ldS<T>(A.diag[dkk(b, +sb)], Qp) / DQ;
        } else {
            cP[k] = T(0);
            cQ[k] = T(0);
        }
        bP[k] = rp / DP;
        bQ[k] = rq / DQ;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        T xp = T(0), xq = T(0);
        for (int k = 0; k < nb; ++k) {
            const T ep = bP[k] + cP[k] * xp, eq = bQ[k] + cQ[k] * xq;
            const T m1 = mPQ[k], m2 = mQP[k];
            const T det = T(1) - m1 * m2;
            xp = (ep + m1 * eq) / det;
            xq = (eq + m2 * ep) / det;
            bP[k] = xp;
            bQ[k] = xq;
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        A.out[gidx(len[a] - 1, k)] = (TOUT)bP[k];
        A.out[gidx(len[a], k)] = (TOUT)bQ[k];
    }
}

// ------------------------------------------------------------------ launchers
size_t fast2d_lds_bytes(int lx, int ly, int R, size_t elem) {
    int pitch = lx + 2;
    if ((R * pitch) & 1) ++pitch;
    return elem * ((size_t)(ly + 2) * pitch + 3 * (size_t)(lx + ly) + 3);
}

hipError_t launch_pack2d(const PassGeom &g, Store s, int R, bool transposed, const double *const *diag,
                         const double *piv, const int64_t *toff, const int64_t *foff, void *s_inv, void *s_ax,
                         void *s_ay, void *face, hipStream_t st) {
    Fast2dDiag dg{};
    for (int k = 0; k < 5; ++k) dg.d[k] = diag[k];
    dim3 grid(g.ntiles), blk(256);
    if (s == Store::F64)
        hipLaunchKernelGGL(k_pack2d<double>, grid, blk, 0, st, g, R, transposed ? 1 : 0, dg, piv, toff, foff,
                           (double *)s_inv, (double *)s_ax, (double *)s_ay, (double *)face);
    else if (s == Store::F32)
        hipLaunchKernelGGL(k_pack2d<float>, grid, blk, 0, st, g, R, transposed ? 1 : 0, dg, piv, toff, foff,
                           (float *)s_inv, (float *)s_ax, (float *)s_ay, (float *)face);
    else
        hipLaunchKernelGGL(k_pack2d<uint16_t>, grid, blk, 0, st, g, R, transposed ? 1 : 0, dg, piv, toff, foff,
                           (uint16_t *)s_inv, (uint16_t *)s_ax, (uint16_t *)s_ay, (uint16_t *)face);
    return hipGetLastError();
}

template <int R, typename T, typename S, typename TIN, typename TOUT>
static hipError_t fast_impl(const Fast2dPass &p, const void *in, bool scale_by_piv, void *out, double cscale,
                            hipStream_t st) {
    Fast2dArgs<S, TIN, TOUT> A{};
    A.g = p.g;
    A.s_inv = (const S *)p.s_inv;
    A.s_ax = (const S *)p.s_ax;
    A.s_ay = (const S *)p.s_ay;
    A.face = (const S *)p.face;
    A.toff = p.toff;
    A.foff = p.foff;
    A.in = (const TIN *)in;
    A.out = (TOUT *)out;
    A.scale_by_piv = scale_by_piv ? 1 : 0;
    A.coupled = p.coupled ? 1 : 0;
    A.cscale = cscale;
    size_t sm = fast2d_lds_bytes(p.lxmax, p.lymax, R, sizeof(T));
    hipLaunchKernelGGL((k_fast2d<R, T, S, TIN, TOUT>), dim3(p.g.ntiles), dim3(256), sm, st, A);
    return hipGetLastError();
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t fast_r(const Fast2dPass &p, const void *in, bool scale, void *out, double cs, hipStream_t st) {
    if (p.R == 1) return fast_impl<1, T, S, TIN, TOUT>(p, in, scale, out, cs, st);
    return fast_impl<2, T, S, TIN, TOUT>(p, in, scale, out, cs, st);
}

hipError_t launch_fast2d(const Fast2dPass &p, Store s, const void *in, bool in_f64, bool scale_by_piv, void *out,
                         bool out_f64, double cscale, hipStream_t st) {
    if (s == Store::F64) {
        if (!in_f64 || !out_f64) return hipErrorInvalidValue;
        return fast_r<double, double, double, double>(p, in, scale_by_piv, out, cscale, st);
    }
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return fast_r<float, float, double, float>(p, in, scale_by_piv, out, cscale, st);
        if (!in_f64 && out_f64) return fast_r<float, float, float, double>(p, in, scale_by_piv, out, cscale, st);
        if (in_f64 && out_f64) return fast_r<float, float, double, double>(p, in, scale_by_piv, out, cscale, st);
        return fast_r<float, float, float, float>(p, in, scale_by_piv, out, cscale, st);
    }
    if (in_f64 && !out_f64) return fast_r<float, uint16_t, double, float>(p, in, scale_by_piv, out, cscale, st);
    if (!in_f64 && out_f64) return fast_r<float, uint16_t, float, double>(p, in, scale_by_piv, out, cscale, st);
    if (in_f64 && out_f64) return fast_r<float, uint16_t, double, double>(p, in, scale_by_piv, out, cscale, st);
    return fast_r<float, uint16_t, float, float>(p, in, scale_by_piv, out, cscale, st);
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t endf_impl(const PassGeom &g, const void *const *diag, const void *piv, const void *in, bool scale,
                            void *out, int facemax, hipStream_t st) {
    EndFaceArgs<T, S, TIN, TOUT> A{};
    A.g = g;
    for (int k = 0; k < 5; ++k) A.diag[k] = (const S *)diag[k];
    A.piv = (const S *)piv;
    A.in = (const TIN *)in;
    A.scale_by_piv = scale ? 1 : 0;
    A.out = (TOUT *)out;
    size_t sm = sizeof(T) * 6 * (size_t)facemax;
    hipLaunchKernelGGL((k_end_faces2d_fast<T, S, TIN, TOUT>), dim3(g.ntiles * 2), dim3(64), sm, st, A);
    return hipGetLastError();
}

hipError_t launch_end_faces2d_fast(const PassGeom &g, Store s, const void *const *diag, const void *piv,
                                   const void *in, bool in_f64, bool scale_by_piv, void *out, bool out_f64,
                                   int facemax, hipStream_t st) {
    if (s == Store::F64) return endf_impl<double, double, double, double>(g, diag, piv, in, scale_by_piv, out, facemax, st);
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return endf_impl<float, float, double, float>(g, diag, piv, in, scale_by_piv, out, facemax, st);
        if (!in_f64 && !out_f64) return endf_impl<float, float, float, float>(g, diag, piv, in, scale_by_piv, out, facemax, st);
        if (in_f64 && out_f64) return endf_impl<float, float, double, double>(g, diag, piv, in, scale_by_piv, out, facemax, st);
        return endf_impl<float, float, float, double>(g, diag, piv, in, scale_by_piv, out, facemax, st);
    }
    if (in_f64 && !out_f64) return endf_impl<float, uint16_t, double, float>(g, diag, piv, in, scale_by_piv, out, facemax, st);
    if (!in_f64 && !out_f64) return endf_impl<float, uint16_t, float, float>(g, diag, piv, in, scale_by_piv, out, facemax, st);
    if (in_f64 && out_f64) return endf_impl<float, uint16_t, double, double>(g, diag, piv, in, scale_by_piv, out, facemax, st);
    return endf_impl<float, uint16_t, float, double>(g, diag, piv, in, scale_by_piv, out, facemax, st);
}

} // namespace psw
