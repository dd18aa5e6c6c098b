// psw_fast2d.hip -- wavefront-pipelined 2D half-sweep kernels for gfx950.
//
// One workgroup per tile.  The tile is swept in its local orientation
// (towards +x, +y).  One 64-lane wave carries the recurrence: lane j owns R
// consecutive rows and handles column x = s - j at step s, so each step is a
// whole anti-diagonal of the tile (the frontal sweep of Sec. 3) and lane j
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

#include <algorithm>

namespace psw {

// global-memory (address space 1) object type
template <typename T> using GP = __attribute__((address_space(1))) T;

namespace {

__device__ __forceinline__ float bf16f(uint16_t b) { return bf16_to_f32(b); }

template <typename S> __device__ __forceinline__ S from_f64(double v);
template <> __device__ __forceinline__ double from_f64<double>(double v) { return v; }
template <> __device__ __forceinline__ float from_f64<float>(double v) { return (float)v; }
template <> __device__ __forceinline__ uint16_t from_f64<uint16_t>(double v) { return f64_to_bf16(v); }

template <typename T, typename S> __device__ __forceinline__ T cvt(S v);
template <> __device__ __forceinline__ double cvt<double, double>(double v) { return v; }
template <> __device__ __forceinline__ float cvt<float, float>(float v) { return v; }
template <> __device__ __forceinline__ float cvt<float, double>(double v) { return (float)v; }
template <> __device__ __forceinline__ double cvt<double, float>(float v) { return (double)v; }
template <> __device__ __forceinline__ float cvt<float, uint16_t>(uint16_t v) { return bf16f(v); }

__device__ __forceinline__ double fmadd(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float fmadd(float a, float b, float c) { return __fmaf_rn(a, b, c); }

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

__device__ __forceinline__ Frame2 frame2n(const int sig[2], int n0, int n1, const TileDesc &td) {
    Frame2 f;
    f.d0 = sig[0] * (td.par[0] ? -1 : 1);
    f.d1 = sig[1] * (td.par[1] ? -1 : 1);
    f.lx = td.len[0];
    f.ly = td.len[1];
    f.lox = td.lo[0];
    f.loy = td.lo[1];
    f.cx = f.d0 > 0 ? td.lo[0] > 0 : td.lo[0] + td.len[0] < n0;
    f.cy = f.d1 > 0 ? td.lo[1] > 0 : td.lo[1] + td.len[1] < n1;
    return f;
}

// global coordinate of local coordinate l (l = -1 is the partner across the start face)
__device__ __forceinline__ int gx_of(const Frame2 &f, int x) { return f.d0 > 0 ? f.lox + x : f.lox + f.lx - 1 - x; }
__device__ __forceinline__ int gy_of(const Frame2 &f, int y) { return f.d1 > 0 ? f.loy + y : f.loy + f.ly - 1 - y; }

} // namespace

// ------------------------------------------------------------------ packing
// Coefficients of one pass in compact sweep-major order: step t = x + j of
// lane j (rows R*j .. R*j+R-1) holds the lanes jlo(t)..jhi(t) that have a
// point at that step, R values per lane, followed by 64 zero lane slots.
// Also the partner data of the coupled start faces.  transposed: the
// couplings are those of the upstream neighbour towards the point (a_{R->P})
// and no face is coupled.

// first lane slot of step t: the number of (column, lane) pairs at earlier steps
__host__ __device__ __forceinline__ int64_t fast2d_step_base(int t, int lx, int L) {
    const int64_t a = t <= L ? (int64_t)t * (t + 1) / 2 : (int64_t)L * (L + 1) / 2 + (int64_t)(t - L) * L;
    const int64_t b = t <= lx ? 0 : (int64_t)(t - lx) * (t - lx + 1) / 2;
    return a - b;
}

template <typename S>
__device__ void pack2d_body(const Frame2 &F, int n0, int R, int transposed, const Fast2dDiag &dg,
                            const double *__restrict__ piv, S *s_inv, S *s_ax, S *s_ay, S *fc) {
    const bool cx = !transposed && F.cx, cy = !transposed && F.cy;
    const int L = (F.ly + R - 1) / R;
    const int64_t npairs = (int64_t)F.lx * L;
    for (int64_t q = threadIdx.x; q < npairs + 64; q += blockDim.x) {
        int64_t slot;
        int x = 0, j = 0;
        if (q < npairs) {
            j = (int)(q / F.lx);
            x = (int)(q - (int64_t)j * F.lx);
            const int t = x + j;
            slot = fast2d_step_base(t, F.lx, L) + (j - max(0, t - F.lx + 1));
        } else {
            slot = q; // the zero slots after the last step
        }
        for (int r = 0; r < R; ++r) {
            double inv = 0, ax = 0, ay = 0;
            const int y = R * j + r;
            if (q < npairs && y < F.ly) {
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
            s_inv[slot * R + r] = from_f64<S>(inv);
            s_ax[slot * R + r] = from_f64<S>(ax);
            s_ay[slot * R + r] = from_f64<S>(ay);
        }
    }
    // partner data of the coupled start faces, per row (x face) / column (y face):
    // [1/Piv_Q, a'_{Q->P}, a'_{Q->upstream along the face}, 1/(1 - a'_{P->Q} a'_{Q->P})]
    for (int y = threadIdx.x; y < F.ly; y += blockDim.x) {
        double v0 = 0, v1 = 0, v2 = 0, v3 = 1;
        if (cx) {
            const int gx = gx_of(F, -1), gy = gy_of(F, y);
            const int64_t Q = lin2(n0, gx, gy), P = lin2(n0, gx_of(F, 0), gy);
            v0 = 1.0 / piv[Q];
            v1 = dg.d[dkk(0, +F.d0)][Q] * v0;
            if (y > 0 || cy) v2 = dg.d[dkk(1, -F.d1)][Q] * v0;
            const double apq = dg.d[dkk(0, -F.d0)][P] / piv[P];
            v3 = 1.0 / (1.0 - apq * v1);
        }
        fc[4 * y + 0] = from_f64<S>(v0);
        fc[4 * y + 1] = from_f64<S>(v1);
        fc[4 * y + 2] = from_f64<S>(v2);
        fc[4 * y + 3] = from_f64<S>(v3);
    }
    S *fr = fc + 4 * F.ly;
    for (int x = threadIdx.x; x < F.lx; x += blockDim.x) {
        double v0 = 0, v1 = 0, v2 = 0, v3 = 1;
        if (cy) {
            const int gx = gx_of(F, x), gy = gy_of(F, -1);
            const int64_t Q = lin2(n0, gx, gy), P = lin2(n0, gx, gy_of(F, 0));
            v0 = 1.0 / piv[Q];
            v1 = dg.d[dkk(1, +F.d1)][Q] * v0;
            if (x > 0 || cx) v2 = dg.d[dkk(0, -F.d0)][Q] * v0;
            const double apq = dg.d[dkk(1, -F.d1)][P] / piv[P];
            v3 = 1.0 / (1.0 - apq * v1);
        }
        fr[4 * x + 0] = from_f64<S>(v0);
        fr[4 * x + 1] = from_f64<S>(v1);
        fr[4 * x + 2] = from_f64<S>(v2);
        fr[4 * x + 3] = from_f64<S>(v3);
    }
    if (threadIdx.x == 0) {
        S *fk = fr + 4 * F.lx;
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

template <typename S>
__global__ void k_pack2d(PassGeom g, int R, int transposed, Fast2dDiag dg, const double *__restrict__ piv,
                         const int64_t *__restrict__ toff, const int64_t *__restrict__ foff, S *s_inv, S *s_ax,
                         S *s_ay, S *face) {
    const TileDesc td = g.tiles[blockIdx.x];
    const Frame2 F = frame2(g, td);
    const int64_t t = toff[blockIdx.x];
    pack2d_body<S>(F, g.n[0], R, transposed, dg, piv, s_inv + t, s_ax + t, s_ay + t, face + foff[blockIdx.x]);
}

// ------------------------------------------------------------------ the pipelined half-sweep
template <typename S, typename TIN, typename TOUT> struct Fast2dArgs {
    PassGeom g;
    const S *s_inv, *s_ax, *s_ay, *face;
    const int64_t *toff, *foff;
    const int *otab;
    const int64_t *ooff;
    const TIN *in;
    TOUT *out;
    double cscale;
    const double *add; // optional: out = 0.5 * (cscale * result) + cadd * add
    double cadd;
};

// value of lane j-1 in lane j and 0 in lane 0: one DPP wave shift per 32 bits
// (bound_ctrl writes 0 where there is no source lane)
__device__ __forceinline__ float lane_up(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double lane_up(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffff), 0x138, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), 0x138, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

constexpr int kBufCfg = 0x00020000; // gfx9 buffer resource word 3
constexpr int kPf = 4;              // steps by which right-hand sides and face records are read ahead

// raw buffer load of one lane slot (R values of type S): vector offset voff, scalar offset soff
template <typename V> __device__ __forceinline__ V ldbuf(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ double2 ldbuf<double2>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
template <> __device__ __forceinline__ double ldbuf<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float2 ldbuf<float2>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ float ldbuf<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ uint32_t ldbuf<uint32_t>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
}
template <> __device__ __forceinline__ uint16_t ldbuf<uint16_t>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
}

// LDS pitch (elements) of the tile: at least lx + 2, and such that the
// anti-diagonal accesses of the wave (stride R * pitch - 1) hit distinct banks
__host__ __device__ __forceinline__ int fast2d_pitch(int lx, int R) {
    int p = lx + 2;
    if (((R * p - 1) & 1) == 0) ++p;
    return p;
}

// The two coupled start faces of a start-coupled pass, each a chain of 2x2
// blocks: the y face pairs P = (x, 0) with Q = (x, -1) along x, the x face
// pairs P = (0, y) with Q = (-1, y) along y (eq. 2d:sor2b2; the cross point
// (0,0) with its three partners is the 4x4 block of eq. 2d:sor4b4 and starts
// both chains).  A face chain involves no other point of the tile, so one
// wave solves it before the sweep: every element is the affine map
//   bq = rq + a_qu vQ',  vP = idt (rhs + a_own vP' + a_cross bq),  vQ = bq + a_qp vP
// of the previous element's (vP', vQ'); each lane composes the maps of a
// contiguous chunk, a shuffle scan over the lanes gives each chunk its
// starting state, and the chunk is then stepped through in order.  vP of
// element i is written to fix[i].
template <typename T> struct Aff2 {
    T a00, a01, a10, a11, u0, u1;
};

// l after e
template <typename T> __device__ __forceinline__ Aff2<T> aff_compose(const Aff2<T> &l, const Aff2<T> &e) {
    Aff2<T> n;
    n.a00 = l.a00 * e.a00 + l.a01 * e.a10;
    n.a01 = l.a00 * e.a01 + l.a01 * e.a11;
    n.a10 = l.a10 * e.a00 + l.a11 * e.a10;
    n.a11 = l.a10 * e.a01 + l.a11 * e.a11;
    n.u0 = l.a00 * e.u0 + l.a01 * e.u1 + l.u0;
    n.u1 = l.a10 * e.u0 + l.a11 * e.u1 + l.u1;
    return n;
}

__device__ __forceinline__ float shfl_up1(float v, int d) { return __shfl_up(v, d); }
__device__ __forceinline__ double shfl_up1(double v, int d) { return __shfl_up(v, d); }

template <typename T> __device__ __forceinline__ Aff2<T> aff_shfl_up(const Aff2<T> &a, int d) {
    Aff2<T> r;
    r.a00 = shfl_up1(a.a00, d);
    r.a01 = shfl_up1(a.a01, d);
    r.a10 = shfl_up1(a.a10, d);
    r.a11 = shfl_up1(a.a11, d);
    r.u0 = shfl_up1(a.u0, d);
    r.u1 = shfl_up1(a.u1, d);
    return r;
}

// Data of chain element i: rhs of P, coupling along the chain, coupling to the
// partner, and the partner record (rq = 1/Piv_Q r_Q or r_Q, a_qp, a_qu, idt).
template <typename T> struct ChainEl {
    T rhs, a_own, a_cross, rq, aqp, aqu, idt;
};

template <typename T, typename Get>
__device__ void face_chain(int n, T vp0, T vq0, Get get, T *fix, int lane) {
    constexpr int kKeep = 4; // elements per lane held in registers between the two passes
    const int ch = (n + 63) / 64;
    const int k0 = min(n, lane * ch), k1 = min(n, k0 + ch);
    ChainEl<T> keep[kKeep];
#pragma unroll
    for (int q = 0; q < kKeep; ++q)
        if (k0 + q < k1) keep[q] = get(k0 + q);
    Aff2<T> m{T(1), T(0), T(0), T(1), T(0), T(0)};
    for (int k = k0; k < k1; ++k) {
        ChainEl<T> e;
        if (k - k0 < kKeep) {
#pragma unroll
            for (int q = 0; q < kKeep; ++q)
                if (q == k - k0) e = keep[q];
        } else {
            e = get(k);
        }
        Aff2<T> a;
        a.a00 = e.idt * e.a_own;
        a.a01 = e.idt * e.a_cross * e.aqu;
        a.u0 = e.idt * (e.rhs + e.a_cross * e.rq);
        a.a10 = e.aqp * a.a00;
        a.a11 = e.aqu + e.aqp * a.a01;
        a.u1 = e.rq + e.aqp * a.u0;
        m = aff_compose(a, m);
    }
    for (int d = 1; d < 64; d <<= 1) {
        const Aff2<T> o = aff_shfl_up(m, d);
        if (lane >= d) m = aff_compose(m, o);
    }
    const Aff2<T> prev = aff_shfl_up(m, 1);
    T vp = vp0, vq = vq0;
    if (lane > 0) {
        vp = prev.a00 * vp0 + prev.a01 * vq0 + prev.u0;
        vq = prev.a10 * vp0 + prev.a11 * vq0 + prev.u1;
    }
    for (int k = k0; k < k1; ++k) {
        ChainEl<T> e;
        if (k - k0 < kKeep) {
#pragma unroll
            for (int q = 0; q < kKeep; ++q)
                if (q == k - k0) e = keep[q];
        } else {
            e = get(k);
        }
        const T bq = e.rq + e.aqu * vq;
        const T np = e.idt * (e.rhs + e.a_own * vp + e.a_cross * bq);
        vq = bq + e.aqp * np;
        vp = np;
        fix[k] = np;
    }
}

// One tile of a pass.  The tile is swept in local orientation (towards +x,
// +y); the LDS copy of the input tile uses local coordinates too.
//   wave 0     : the recurrence, kFast2dBlk anti-diagonal steps per barrier
//                interval; lane j owns rows R*j .. R*j+R-1 and handles column
//                x = s - j at step s; the row above arrives by a DPP shift.
//   waves 1..3 : stage column block i + 2 and write back column block i - lag
//                (all of whose points are final) during interval i; before
//                the sweep, waves 1 and 2 solve the coupled start faces.
// Coefficients stream from the compact sweep-major packing through a
// register ring of RING steps; the right-hand sides come from LDS kPf steps
// ahead.  Lanes without a point at a step compute with another slot's
// coefficients and finite LDS values; their results reach no lane that has a
// point and are written to a per-lane sink.
template <int R, typename T, typename S, typename TIN, typename TOUT, bool SC, bool CPL>
__device__ __forceinline__ void fast2d_body(const Frame2 &F, int n0, const GP<TIN> *__restrict__ in,
                                            GP<TOUT> *__restrict__ out, const S *s_inv_t, const S *s_ax_t,
                                            const S *s_ay_t, const GP<int> *__restrict__ tab, const GP<S> *fsrc,
                                            double cscale, const GP<double> *__restrict__ add, double cadd,
                                            unsigned char *smem) {
    using V = typename Pack<S, R>::V;
    constexpr int RING = SC ? 16 : 8;
    constexpr int KB = kFast2dBlk;
    const bool cx = CPL && F.cx, cy = CPL && F.cy;
    const int lx = F.lx, ly = F.ly;
    const int L = (ly + R - 1) / R;
    const int nsteps = lx + L - 1;
    const int niter = (nsteps + KB - 1) / KB;
    const int nblk = (lx + KB - 1) / KB;
    const int lag = (L + KB - 2) / KB + 1; // block c is final after interval c + lag - 1
    const int pitch = fast2d_pitch(lx, R);
    T *vt = reinterpret_cast<T *>(smem);
    const int sink = (ly + 2) * pitch; // 64 + (R - 1) * pitch sink slots
    T *yfix = vt + sink + 64 + pitch;  // solved y-face points (x, 0)
    T *xfix = yfix + lx;               // solved x-face points (0, y)
    const int tid = threadIdx.x;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;

    // ---- borders: zero column -1 and lx, row -1 and ly (partners are read from memory by the face chains)
    for (int r = tid; r < ly + 2; r += 256) {
        vt[r * pitch] = T(0);
        vt[r * pitch + lx + 1] = T(0);
    }
    for (int c = tid; c < lx; c += 256) {
        vt[c + 1] = T(0);
        vt[(ly + 1) * pitch + c + 1] = T(0);
    }

    // ---- staging / write-back of column blocks by waves 1..3
    constexpr int NH = 192;
    constexpr int NB = (128 * KB + NH - 1) / NH;
    const int ht = tid - 64;
    auto stage = [&](int b) {
        const int c0 = b * KB, nc = min(KB, lx - c0);
        T v[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = ht + NH * u;
            const int y = e / KB, c = e - y * KB;
            v[u] = (y < ly && c < nc) ? cvt<T>(in[lin2(n0, gx_of(F, c0 + c), gy_of(F, y))]) : T(0);
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = ht + NH * u;
            const int y = e / KB, c = e - y * KB;
            if (y < ly && c < nc) vt[(y + 1) * pitch + c0 + c + 1] = v[u];
        }
    };
    const T cs = (T)cscale;
    auto wback = [&](int b) {
        const int c0 = b * KB, nc = min(KB, lx - c0);
        T v[NB];
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = ht + NH * u;
            const int y = e / KB, c = e - y * KB;
            v[u] = (y < ly && c < nc) ? vt[(y + 1) * pitch + c0 + c + 1] : T(0);
        }
        if (add) {
            // the symmetric combination: 0.5 * (cscale * result) + cadd * add, in FP64;
            // all addends are loaded before the first store
            double av[NB];
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int e = ht + NH * u;
                const int y = e / KB, c = e - y * KB;
                av[u] = (y < ly && c < nc) ? add[lin2(n0, gx_of(F, c0 + c), gy_of(F, y))] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < NB; ++u) {
                const int e = ht + NH * u;
                const int y = e / KB, c = e - y * KB;
                if (y < ly && c < nc)
                    out[lin2(n0, gx_of(F, c0 + c), gy_of(F, y))] = (TOUT)(0.5 * (double)(cs * v[u]) + cadd * av[u]);
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < NB; ++u) {
            const int e = ht + NH * u;
            const int y = e / KB, c = e - y * KB;
            if (y < ly && c < nc) out[lin2(n0, gx_of(F, c0 + c), gy_of(F, y))] = (TOUT)(cs * v[u]);
        }
    };
    const int nbytes = tab[0];
    if (wv >= 1) {
        stage(0);
        if (nblk > 1) stage(1);
    }
    if (CPL && (wv == 1 || wv == 2) && (wv == 1 ? cy : cx)) {
        // ---- coupled start faces (wave 1: y face, wave 2: x face)
        const GP<S> *ci = (const GP<S> *)s_inv_t, *cax = (const GP<S> *)s_ax_t, *cay = (const GP<S> *)s_ay_t;
        // packed coefficients of local point (x, y): lane j = y / R, element y % R of step x + j
        auto coef = [&](int x, int y, T &iv, T &ax, T &ay) {
            const int j = y / R, t = x + j;
            const int64_t e = (fast2d_step_base(t, lx, L) + j - max(0, t - lx + 1)) * R + (y - j * R);
            iv = SC ? T(1) : cvt<T>(ci[e]);
            ax = cvt<T>(cax[e]);
            ay = cvt<T>(cay[e]);
        };
        auto rhs_of = [&](T iv, T r) -> T { return SC ? r : iv * r; };
        auto inv_at = [&](int x, int y) -> T { return cvt<T>(in[lin2(n0, gx_of(F, x), gy_of(F, y))]); };
        const GP<S> *fxr = fsrc, *fyr = fsrc + 4 * ly, *fkr = fsrc + 4 * (lx + ly);
        // cross point: A = (0,0), B = (-1,0), C = (0,-1), D = (-1,-1)
        T vA = T(0), vB = T(0), vC = T(0);
        if (cx && cy) {
            T iv, ax, ay;
            coef(0, 0, iv, ax, ay);
            const T rhs = rhs_of(iv, inv_at(0, 0));
            const T ivq = cvt<T>(fxr[0]), aqp = cvt<T>(fxr[1]), aqy = cvt<T>(fxr[2]);
            const T ivc = cvt<T>(fyr[0]), acp = cvt<T>(fyr[1]), acd = cvt<T>(fyr[2]);
            const T ivd = cvt<T>(fkr[0]), adb = cvt<T>(fkr[1]), adc = cvt<T>(fkr[2]);
            const T rq = rhs_of(ivq, inv_at(-1, 0)), rcc = rhs_of(ivc, inv_at(0, -1)), rd = rhs_of(ivd, inv_at(-1, -1));
            T M[4][4] = {{T(1), -ax, -ay, T(0)}, {-aqp, T(1), T(0), -aqy}, {-acp, T(0), T(1), -acd}, {T(0), -adb, -adc, T(1)}};
            T bb[4] = {rhs, rq, rcc, rd};
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const T ip = T(1) / M[p][p];
#pragma unroll
                for (int i = p + 1; i < 4; ++i) {
                    const T l = M[i][p] * ip;
#pragma unroll
                    for (int jj = p + 1; jj < 4; ++jj) M[i][jj] -= l * M[p][jj];
                    bb[i] -= l * bb[p];
                }
            }
#pragma unroll
            for (int i = 3; i >= 0; --i) {
                T acc = bb[i];
#pragma unroll
                for (int jj = i + 1; jj < 4; ++jj) acc -= M[i][jj] * bb[jj];
                bb[i] = acc / M[i][i];
            }
            vA = bb[0];
            vB = bb[1];
            vC = bb[2];
        }
        const int first = (cx && cy) ? 1 : 0; // the cross point is the chains' element 0
        if (wv == 1) {
            if (first && lane == 0) yfix[0] = vA;
            face_chain<T>(
                lx - first, vA, vC,
                [&](int k) {
                    const int x = k + first;
                    ChainEl<T> e;
                    T iv;
                    coef(x, 0, iv, e.a_own, e.a_cross);
                    e.rhs = rhs_of(iv, inv_at(x, 0));
                    const T ivq = cvt<T>(fyr[4 * x]);
                    e.aqp = cvt<T>(fyr[4 * x + 1]);
                    e.aqu = cvt<T>(fyr[4 * x + 2]);
                    e.idt = cvt<T>(fyr[4 * x + 3]);
                    e.rq = rhs_of(ivq, inv_at(x, -1));
                    return e;
                },
                yfix + first, lane);
        } else {
            if (first && lane == 0) xfix[0] = vA;
            face_chain<T>(
                ly - first, vA, vB,
                [&](int k) {
                    const int y = k + first;
                    ChainEl<T> e;
                    T iv;
                    coef(0, y, iv, e.a_cross, e.a_own);
                    e.rhs = rhs_of(iv, inv_at(0, y));
                    const T ivq = cvt<T>(fxr[4 * y]);
                    e.aqp = cvt<T>(fxr[4 * y + 1]);
                    e.aqu = cvt<T>(fxr[4 * y + 2]);
                    e.idt = cvt<T>(fxr[4 * y + 3]);
                    e.rq = rhs_of(ivq, inv_at(-1, y));
                    return e;
                },
                xfix + first, lane);
        }
    }
    __syncthreads();

    // ---- recurrence state (wave 0)
    const int lane_c = min(lane, L - 1);
    const int rowa = (R * lane_c + 1) * pitch + 1; // LDS index of (x = 0, first row of this lane)
    const __amdgpu_buffer_rsrc_t rinv = __builtin_amdgcn_make_buffer_rsrc((void *)s_inv_t, 0, nbytes, kBufCfg);
    const __amdgpu_buffer_rsrc_t rax = __builtin_amdgcn_make_buffer_rsrc((void *)s_ax_t, 0, nbytes, kBufCfg);
    const __amdgpu_buffer_rsrc_t ray = __builtin_amdgcn_make_buffer_rsrc((void *)s_ay_t, 0, nbytes, kBufCfg);
    const int voff = lane * R * (int)sizeof(S);
    V ri[RING], ra[RING], rb[RING];
    T rc[kPf][R]; // right-hand sides of the next kPf steps
    T yf[kPf];    // solved y-face points of the next kPf columns
    T left[R];
    T last = T(0);
    const bool l0 = lane == 0;
#pragma unroll
    for (int r = 0; r < R; ++r) left[r] = T(0);
    T xf[R]; // solved x-face points of this lane's rows
#pragma unroll
    for (int r = 0; r < R; ++r) xf[r] = (CPL && cx) ? xfix[min(R * lane_c + r, ly - 1)] : T(0);
    if (wv == 0) {
#pragma unroll
        for (int k = 0; k < RING; ++k) {
            const int so = tab[1 + k];
            if (!SC) ri[k] = ldbuf<V>(rinv, voff, so);
            ra[k] = ldbuf<V>(rax, voff, so);
            rb[k] = ldbuf<V>(ray, voff, so);
        }
#pragma unroll
        for (int k = 0; k < kPf; ++k) {
            const int x = min(max(k - lane, -1), lx);
#pragma unroll
            for (int r = 0; r < R; ++r) rc[k][r] = vt[rowa + r * pitch + x];
            if (CPL) yf[k] = yfix[min(k, lx - 1)];
        }
    }

    // one step; XF: some lane may be at x = 0; so: offset of the slot read RING steps ahead
    auto step = [&](const int s, const int k, const bool XF, const int so) {
        const int slot = k % RING, pk = k % kPf;
        const int x = s - lane;
        const T up_in = lane_up(last);
        T cur[R];
#pragma unroll
        for (int r = 0; r < R; ++r) cur[r] = rc[pk][r];
        {
            const int xn = min(max(s + kPf - lane, -1), lx);
#pragma unroll
            for (int r = 0; r < R; ++r) rc[pk][r] = vt[rowa + r * pitch + xn];
        }
        // read whether or not the y face is coupled (used only if it is): a branch here
        // would split the unrolled interval into one block per step
        T yv = T(0);
        if (CPL) {
            yv = yf[pk];
            yf[pk] = yfix[min(s + kPf, lx - 1)];
        }
        const bool isx = XF && cx && x == 0;
        T v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const T iv = SC ? T(1) : elem<T>(ri[slot], r);
            const T ax = elem<T>(ra[slot], r), ay = elem<T>(rb[slot], r);
            const T rhs = SC ? cur[r] : iv * cur[r];
            const T u = r == 0 ? up_in : v[r - 1];
            // fused multiply-adds written out, so that the rounding does not depend on how
            // the compiler contracts the unrolled interval
            T val = fmadd(ay, u, fmadd(ax, left[r], rhs));
            if (CPL && cy && r == 0) val = l0 ? yv : val;
            if (XF && cx) val = isx ? xf[r] : val;
            v[r] = val;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) left[r] = v[r];
        last = v[R - 1];
        const bool act = x >= 0 && x < lx && lane < L;
        const int a = act ? rowa + x : sink + lane;
#pragma unroll
        for (int r = 0; r < R; ++r) vt[a + r * pitch] = v[r];
        if (!SC) ri[slot] = ldbuf<V>(rinv, voff, so);
        ra[slot] = ldbuf<V>(rax, voff, so);
        rb[slot] = ldbuf<V>(ray, voff, so);
        // keeps each step's loads in step order, so the ring's loads stay in flight across
        // the interval's end instead of being drained by a wait at the loop head
        __builtin_amdgcn_sched_barrier(0);
    };

    // helper waves: stage block i + 2, write back block i - lag
    auto helpers = [&](int i) {
        if (i + 2 < nblk) stage(i + 2);
        if (i - lag >= 0 && i - lag < nblk) wback(i - lag);
    };
    // Wave 0 and the helper waves run separate loops with one barrier per
    // interval each, so the recurrence state is not live in the helpers' code.
    if (wv == 0) {
        // The slot offsets of an interval are read one interval ahead into scalar
        // registers: a scalar load inside a step would make the step wait for it
        // together with all LDS reads in flight (they share one counter).
        int so_n[KB];
        auto offsets = [&](int i) {
#pragma unroll
            for (int k = 0; k < KB; ++k) so_n[k] = tab[1 + i * KB + k + RING];
        };
        offsets(0);
        // intervals in which some lane meets the x face, then the rest
        const int nxf = (CPL && cx) ? min(niter, (L + KB - 1) / KB) : 0;
        for (int i = 0; i < nxf; ++i) {
            int so[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) so[k] = so_n[k];
            offsets(i + 1);
#pragma unroll
            for (int k = 0; k < KB; ++k) step(i * KB + k, k, CPL, so[k]);
            __syncthreads();
        }
        for (int i = nxf; i < niter; ++i) {
            int so[KB];
#pragma unroll
            for (int k = 0; k < KB; ++k) so[k] = so_n[k];
            offsets(i + 1);
#pragma unroll
            for (int k = 0; k < KB; ++k) step(i * KB + k, k, false, so[k]);
            __syncthreads();
        }
    } else {
        for (int i = 0; i < niter; ++i) {
            helpers(i);
            __syncthreads();
        }
    }
    if (wv >= 1)
        for (int b = max(0, niter - lag); b < nblk; ++b) wback(b);
}

template <int R, typename T, typename S, typename TIN, typename TOUT, bool SC, bool CPL>
__global__ void __launch_bounds__(256) k_fast2d(Fast2dArgs<S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const TileDesc td = A.g.tiles[blockIdx.x];
    const Frame2 F = frame2(A.g, td);
    const int64_t t = A.toff[blockIdx.x];
    fast2d_body<R, T, S, TIN, TOUT, SC, CPL>(F, A.g.n[0], (const GP<TIN> *)A.in, (GP<TOUT> *)A.out, A.s_inv + t,
                                              A.s_ax + t, A.s_ay + t, (const GP<int> *)(A.otab + A.ooff[blockIdx.x]),
                                              (const GP<S> *)(A.face + A.foff[blockIdx.x]), A.cscale,
                                              (const GP<double> *)A.add, A.cadd, smem);
}

// ------------------------------------------------------------------ end-face chains (2D), prefetched
// The coupled end face owned by a tile (see k_end_faces in psw_kernels.hip):
// all data of the chain that does not depend on the chain itself is gathered
// into LDS by the workgroup; one thread then runs the 2x2 recurrence.

template <typename T, typename S> __device__ __forceinline__ T ldS(const GP<S> *p, int64_t i) { return cvt<T>(p[i]); }

// Tile frame of an end-coupled pass on axis pair (a, b).
struct EndFrame2 {
    int d[2], len[2], lo[2];
    bool endc[2];
};

__device__ __forceinline__ EndFrame2 end_frame2(const int sig[2], int n0, int n1, const TileDesc &td) {
    EndFrame2 f;
    const int n[2] = {n0, n1};
    for (int q = 0; q < 2; ++q) {
        f.d[q] = sig[q] * (td.par[q] ? -1 : 1);
        f.len[q] = td.len[q];
        f.lo[q] = td.lo[q];
        f.endc[q] = f.d[q] > 0 ? f.lo[q] + f.len[q] < n[q] : f.lo[q] > 0;
    }
    return f;
}

// The coupled end face on axis A owned by this tile (the tile sweeps towards
// it): all data of the 2x2 chain that does not depend on the chain itself is
// gathered into LDS by the workgroup; one thread then runs the recurrence.
// The axis is a template argument and the diagonals are picked by selects, so
// that no frame array is indexed at run time (that would put it in scratch
// memory, one memory round trip per access).
template <int A, typename T, typename S, typename TIN, typename TOUT>
__device__ void end_face2d_body(const EndFrame2 &E, int n0, const GP<S> *const *diag, const GP<S> *piv,
                                const GP<TIN> *in, bool scale_by_piv, GP<TOUT> *out, unsigned char *smem) {
    constexpr int B = 1 - A;
    const int da = A ? E.d[1] : E.d[0], db = A ? E.d[0] : E.d[1];
    const int lena = A ? E.len[1] : E.len[0], lenb = A ? E.len[0] : E.len[1];
    const int loa = A ? E.lo[1] : E.lo[0], lob = A ? E.lo[0] : E.lo[1];
    const bool endca = A ? E.endc[1] : E.endc[0], endcb = A ? E.endc[0] : E.endc[1];
    if (!(da > 0 && endca)) return;
    const int nb = endcb ? lenb - 1 : lenb;
    T *mPQ = reinterpret_cast<T *>(smem);
    T *mQP = mPQ + nb, *cP = mQP + nb, *cQ = cP + nb, *bP = cQ + nb, *bQ = bP + nb;
    auto gidx = [&](int la, int lb) -> int64_t {
        const int ca = da > 0 ? loa + la : loa + lena - 1 - la;
        const int cb = db > 0 ? lob + lb : lob + lenb - 1 - lb;
        return A == 0 ? (int64_t)ca + (int64_t)n0 * cb : (int64_t)cb + (int64_t)n0 * ca;
    };
    // couplings along axis A towards +da / -da, and along B towards +db (diagonal k = 1 + 2 axis + side)
    const GP<S> *dAp = da > 0 ? diag[2 + 2 * A] : diag[1 + 2 * A];
    const GP<S> *dAm = da > 0 ? diag[1 + 2 * A] : diag[2 + 2 * A];
    const GP<S> *dBp = db > 0 ? diag[2 + 2 * B] : diag[1 + 2 * B];
    // P at local (la = len_a-1, lb), Q at la = len_a (across), inward neighbours at len_a-2 and len_a+1
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        const int64_t P = gidx(lena - 1, k), Q = gidx(lena, k);
        const int64_t Pin = gidx(lena - 2, k), Qin = gidx(lena + 1, k);
        const T DP = ldS<T>(piv, P), DQ = ldS<T>(piv, Q);
        T rp = cvt<T>(in[P]), rq = cvt<T>(in[Q]);
        if (scale_by_piv) {
            rp *= DP;
            rq *= DQ;
        }
        // couplings of the neighbours towards P / Q (transposed rows)
        rp += ldS<T>(dAp, Pin) * cvt<T>(out[Pin]);
        rq += ldS<T>(dAm, Qin) * cvt<T>(out[Qin]);
        const T iP = T(1) / DP, iQ = T(1) / DQ;
        const T m1 = ldS<T>(dAm, Q) * iP; // Q's coupling towards P
        const T m2 = ldS<T>(dAp, P) * iQ; // P's coupling towards Q
        mPQ[k] = m1 / (T(1) - m1 * m2);   // pre-divided by the 2x2 determinant
        mQP[k] = m2;
        if (k > 0) {
            const int64_t Pp = gidx(lena - 1, k - 1), Qp = gidx(lena, k - 1);
            cP[k] = ldS<T>(dBp, Pp) * iP;
            cQ[k] = ldS<T>(dBp, Qp) * iQ;
        } else {
            cP[k] = T(0);
            cQ[k] = T(0);
        }
        bP[k] = rp * iP;
        bQ[k] = rq * iQ;
    }
    __syncthreads();
    // The chain X_k = (x_P, x_Q)_k = A_k X_{k-1} + u_k, X_{-1} = 0, with
    //   e_P = b_P + c_P x_P',  e_Q = b_Q + c_Q x_Q',
    //   x_P = e_P idet + m1d e_Q,  x_Q = e_Q + m2 x_P   (idet = 1 + m1d m2).
    // Each of the 64 threads takes a contiguous chunk of ch entries, composes
    // its chunk's affine maps, a scan over the chunks gives every chunk its
    // starting state, and the chunk is then stepped through in order.
    const int nt = blockDim.x, t = threadIdx.x;
    const int ch = (nb + nt - 1) / nt;
    const int k0 = min(nb, t * ch), k1 = min(nb, k0 + ch);
    T c00 = T(1), c01 = T(0), c10 = T(0), c11 = T(1), c0 = T(0), c1 = T(0); // identity map
    for (int k = k0; k < k1; ++k) {
        const T m1d = mPQ[k], m2 = mQP[k];
        const T idet = T(1) + m1d * m2;
        const T a00 = idet * cP[k], a01 = m1d * cQ[k], a10 = m2 * a00, a11 = idet * cQ[k];
        const T u0 = idet * bP[k] + m1d * bQ[k], u1 = bQ[k] + m2 * u0;
        // new = entry o chunk-so-far
        const T n00 = a00 * c00 + a01 * c10, n01 = a00 * c01 + a01 * c11;
        const T n10 = a10 * c00 + a11 * c10, n11 = a10 * c01 + a11 * c11;
        const T n0 = a00 * c0 + a01 * c1 + u0, n1 = a10 * c0 + a11 * c1 + u1;
        c00 = n00; c01 = n01; c10 = n10; c11 = n11; c0 = n0; c1 = n1;
    }
    // inclusive scan of the chunk maps (Hillis-Steele over the 64 threads)
    T *sc = bQ + nb; // 6 * nt values
    for (int off = 1; off < nt; off <<= 1) {
        sc[6 * t + 0] = c00; sc[6 * t + 1] = c01; sc[6 * t + 2] = c10;
        sc[6 * t + 3] = c11; sc[6 * t + 4] = c0; sc[6 * t + 5] = c1;
        __syncthreads();
        if (t >= off) {
            const T *e = sc + 6 * (t - off);
            const T e00 = e[0], e01 = e[1], e10 = e[2], e11 = e[3], e0 = e[4], e1 = e[5];
            const T n00 = c00 * e00 + c01 * e10, n01 = c00 * e01 + c01 * e11;
            const T n10 = c10 * e00 + c11 * e10, n11 = c10 * e01 + c11 * e11;
            const T n0 = c00 * e0 + c01 * e1 + c0, n1 = c10 * e0 + c11 * e1 + c1;
            c00 = n00; c01 = n01; c10 = n10; c11 = n11; c0 = n0; c1 = n1;
        }
        __syncthreads();
    }
    // state before this chunk = the previous thread's inclusive result applied to X_{-1} = 0
    sc[2 * t] = c0;
    sc[2 * t + 1] = c1;
    __syncthreads();
    T xp = t > 0 ? sc[2 * (t - 1)] : T(0), xq = t > 0 ? sc[2 * (t - 1) + 1] : T(0);
    __syncthreads();
    for (int k = k0; k < k1; ++k) {
        const T ep = bP[k] + cP[k] * xp, eq = bQ[k] + cQ[k] * xq;
        const T m1d = mPQ[k], m2 = mQP[k];
        const T idet = T(1) + m1d * m2;
        xp = ep * idet + m1d * eq;
        xq = eq + m2 * xp;
        bP[k] = xp;
        bQ[k] = xq;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
        out[gidx(lena - 1, k)] = (TOUT)bP[k];
        out[gidx(lena, k)] = (TOUT)bQ[k];
    }
}

// Cross point of two coupled end faces, owned by the tile sweeping towards
// +x and +y: the 4x4 block of the corner points of the four tiles.
template <typename T, typename S, typename TIN, typename TOUT>
__device__ void end_corner2d_body(const EndFrame2 &E, int n0, const GP<S> *const *diag, const GP<S> *piv,
                                  const GP<TIN> *in, bool scale_by_piv, GP<TOUT> *out) {
    if (!(E.d[0] > 0 && E.endc[0] && E.d[1] > 0 && E.endc[1])) return;
    const int gx = E.lo[0] + E.len[0] - 1, gy = E.lo[1] + E.len[1] - 1;
    // block points B = bit0 (x shifted by +1), bit1 (y shifted by +1)
    T M[4][4], R[4];
    int64_t idx[4];
    for (int B = 0; B < 4; ++B) {
        const int qx = gx + (B & 1), qy = gy + ((B >> 1) & 1);
        idx[B] = (int64_t)qx + (int64_t)n0 * qy;
    }
    for (int B = 0; B < 4; ++B) {
        const int fx = B & 1, fy = (B >> 1) & 1;
        const int dqx = fx ? -1 : 1, dqy = fy ? -1 : 1; // direction of the point's own tile
        const int qx = gx + fx, qy = gy + fy;
        const int64_t Q = idx[B];
        const T D = ldS<T>(piv, Q), iD = T(1) / D;
        T acc = cvt<T>(in[Q]);
        if (scale_by_piv) acc *= D;
        for (int j = 0; j < 4; ++j) M[B][j] = (j == B) ? T(1) : T(0);
        // block mates across x and y: their couplings towards Q
        {
            const int s = fx ? -1 : 1; // Q + s e_x is the mate
            M[B][B ^ 1] -= ldS<T>(diag[dkk(0, -s)], idx[B ^ 1]) * iD;
        }
        {
            const int s = fy ? -1 : 1;
            M[B][B ^ 2] -= ldS<T>(diag[dkk(1, -s)], idx[B ^ 2]) * iD;
        }
        // upstream points inside the point's own tile (chain values of the faces)
        {
            const int64_t Rx = (int64_t)(qx - dqx) + (int64_t)n0 * qy;
            acc += ldS<T>(diag[dkk(0, dqx)], Rx) * cvt<T>(out[Rx]);
        }
        {
            const int64_t Ry = (int64_t)qx + (int64_t)n0 * (qy - dqy);
            acc += ldS<T>(diag[dkk(1, dqy)], Ry) * cvt<T>(out[Ry]);
        }
        R[B] = acc * iD;
    }
    for (int k = 0; k < 4; ++k) {
        const T ip = T(1) / M[k][k];
        for (int i = k + 1; i < 4; ++i) {
            const T l = M[i][k] * ip;
            for (int j = k + 1; j < 4; ++j) M[i][j] -= l * M[k][j];
            R[i] -= l * R[k];
        }
    }
    for (int i = 3; i >= 0; --i) {
        T acc = R[i];
        for (int j = i + 1; j < 4; ++j) acc -= M[i][j] * R[j];
        R[i] = acc / M[i][i];
    }
    for (int B = 0; B < 4; ++B) out[idx[B]] = (TOUT)R[B];
}

template <typename T, typename S, typename TIN, typename TOUT> struct EndFaceArgs {
    PassGeom g;
    const S *diag[5];
    const S *piv;
    const TIN *in;
    int scale_by_piv;
    TOUT *out;
};

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(64) k_end_faces2d_fast(EndFaceArgs<T, S, TIN, TOUT> A) {
    extern __shared__ __align__(16) unsigned char smem[];
    const TileDesc td = A.g.tiles[blockIdx.x >> 1];
    const EndFrame2 E = end_frame2(A.g.sig, A.g.n[0], A.g.n[1], td);
    const GP<S> *dg[5] = {(const GP<S> *)A.diag[0], (const GP<S> *)A.diag[1], (const GP<S> *)A.diag[2],
                          (const GP<S> *)A.diag[3], (const GP<S> *)A.diag[4]};
    if (blockIdx.x & 1)
        end_face2d_body<1, T, S, TIN, TOUT>(E, A.g.n[0], dg, (const GP<S> *)A.piv, (const GP<TIN> *)A.in,
                                            A.scale_by_piv != 0, (GP<TOUT> *)A.out, smem);
    else
        end_face2d_body<0, T, S, TIN, TOUT>(E, A.g.n[0], dg, (const GP<S> *)A.piv, (const GP<TIN> *)A.in,
                                            A.scale_by_piv != 0, (GP<TOUT> *)A.out, smem);
}

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void k_end_corners2d(EndFaceArgs<T, S, TIN, TOUT> A) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= A.g.ntiles) return;
    const EndFrame2 E = end_frame2(A.g.sig, A.g.n[0], A.g.n[1], A.g.tiles[t]);
    const GP<S> *dg[5] = {(const GP<S> *)A.diag[0], (const GP<S> *)A.diag[1], (const GP<S> *)A.diag[2],
                          (const GP<S> *)A.diag[3], (const GP<S> *)A.diag[4]};
    end_corner2d_body<T, S, TIN, TOUT>(E, A.g.n[0], dg, (const GP<S> *)A.piv, (const GP<TIN> *)A.in,
                                       A.scale_by_piv != 0, (GP<TOUT> *)A.out);
}

// ------------------------------------------------------------------ launchers
void fast2d_fill_tab(int lx, int ly, int R, size_t elem, int *tab) {
    const int L = (ly + R - 1) / R, nsteps = lx + L - 1;
    const int n = fast2d_tab_len(lx, ly, R);
    tab[0] = (int)(fast2d_tile_elems(lx, ly, R, elem) * (int64_t)elem);
    const int64_t end = (int64_t)lx * L;
    for (int t = 0; t < n - 1; ++t) {
        const int64_t slot = t < nsteps ? fast2d_step_base(t, lx, L) - std::max(0, t - lx + 1) : end;
        tab[1 + t] = (int)(slot * R * (int64_t)elem);
    }
}

size_t fast2d_lds_bytes(int lx, int ly, int R, size_t elem) {
    const int pitch = fast2d_pitch(lx, R);
    const size_t sink = (size_t)(ly + 2) * pitch;
    return elem * (sink + 64 + pitch + (size_t)(lx + ly));
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

template <int R, typename T, typename S, typename TIN, typename TOUT, bool SC, bool CPL>
static hipError_t fast_impl(const Fast2dPass &p, const void *in, bool scale_by_piv, void *out, double cscale,
                            const double *add, double cadd, hipStream_t st) {
    Fast2dArgs<S, TIN, TOUT> A{};
    A.g = p.g;
    A.s_inv = (const S *)p.s_inv;
    A.s_ax = (const S *)p.s_ax;
    A.s_ay = (const S *)p.s_ay;
    A.face = (const S *)p.face;
    A.toff = p.toff;
    A.foff = p.foff;
    A.otab = p.otab;
    A.ooff = p.ooff;
    A.in = (const TIN *)in;
    A.out = (TOUT *)out;
    A.cscale = cscale;
    A.add = add;
    A.cadd = cadd;
    size_t sm = fast2d_lds_bytes(p.lxmax, p.lymax, R, sizeof(T));
    hipLaunchKernelGGL((k_fast2d<R, T, S, TIN, TOUT, SC, CPL>), dim3(p.g.ntiles), dim3(256), sm, st, A);
    return hipGetLastError();
}

template <int R, typename T, typename S, typename TIN, typename TOUT>
static hipError_t fast_flags(const Fast2dPass &p, const void *in, bool scale, void *out, double cs, const double *add,
                             double cadd, hipStream_t st) {
    if (scale) {
        if (p.coupled) return fast_impl<R, T, S, TIN, TOUT, true, true>(p, in, scale, out, cs, add, cadd, st);
        return fast_impl<R, T, S, TIN, TOUT, true, false>(p, in, scale, out, cs, add, cadd, st);
    }
    if (p.coupled) return fast_impl<R, T, S, TIN, TOUT, false, true>(p, in, scale, out, cs, add, cadd, st);
    return fast_impl<R, T, S, TIN, TOUT, false, false>(p, in, scale, out, cs, add, cadd, st);
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t fast_r(const Fast2dPass &p, const void *in, bool scale, void *out, double cs, const double *add,
                         double cadd, hipStream_t st) {
    if (p.R == 1) return fast_flags<1, T, S, TIN, TOUT>(p, in, scale, out, cs, add, cadd, st);
    return fast_flags<2, T, S, TIN, TOUT>(p, in, scale, out, cs, add, cadd, st);
}

hipError_t launch_fast2d(const Fast2dPass &p, Store s, const void *in, bool in_f64, bool scale_by_piv, void *out,
                         bool out_f64, double cscale, const double *add, double cadd, hipStream_t st) {
    if (add && !out_f64) return hipErrorInvalidValue;
#define PSW_F_ARGS p, in, scale_by_piv, out, cscale, add, cadd, st
    if (s == Store::F64) {
        if (!in_f64 || !out_f64) return hipErrorInvalidValue;
        return fast_r<double, double, double, double>(PSW_F_ARGS);
    }
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return fast_r<float, float, double, float>(PSW_F_ARGS);
        if (!in_f64 && out_f64) return fast_r<float, float, float, double>(PSW_F_ARGS);
        if (in_f64 && out_f64) return fast_r<float, float, double, double>(PSW_F_ARGS);
        return fast_r<float, float, float, float>(PSW_F_ARGS);
    }
    if (in_f64 && !out_f64) return fast_r<float, uint16_t, double, float>(PSW_F_ARGS);
    if (!in_f64 && out_f64) return fast_r<float, uint16_t, float, double>(PSW_F_ARGS);
    if (in_f64 && out_f64) return fast_r<float, uint16_t, double, double>(PSW_F_ARGS);
    return fast_r<float, uint16_t, float, float>(PSW_F_ARGS);
#undef PSW_F_ARGS
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
    size_t sm = sizeof(T) * 6 * ((size_t)facemax + 64); // chain data + scan area of 64 threads
    hipLaunchKernelGGL((k_end_faces2d_fast<T, S, TIN, TOUT>), dim3(g.ntiles * 2), dim3(64), sm, st, A);
    hipLaunchKernelGGL((k_end_corners2d<T, S, TIN, TOUT>), dim3((g.ntiles + 63) / 64), dim3(64), 0, st, A);
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

// ------------------------------------------------------------------ batched 2D passes
// Pointers read from the problem table are generic; casting them through the
// global address space lets the compiler emit global (not flat) memory
// instructions, which do not hold up the LDS counters.
template <typename T> __device__ __forceinline__ GP<T> *as_global(const void *p) {
    return (GP<T> *)p;
}

__device__ __forceinline__ void *bslot(const BProb &P, int k) { return P.vec[k]; }

template <int R, typename T, typename S, typename TIN, typename TOUT, bool SC, bool CPL>
__global__ void __launch_bounds__(256) k_b_fast2d(const BTile *__restrict__ tiles, const BProb *__restrict__ probs, int sig0, int sig1,
                                                  int pass, int in_slot, int out_slot, int cs_from_prob, int add_slot) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BTile tb = tiles[blockIdx.x];
    const BProb &P = probs[tb.prob];
    if (P.flags[0] == 0) return;
    const int sig[2] = {sig0, sig1};
    const Frame2 F = frame2n(sig, P.n0, P.n1, tb.td);
    const int64_t t = P.toff[tb.tix];
    fast2d_body<R, T, S, TIN, TOUT, SC, CPL>(
        F, P.n0, as_global<const TIN>(bslot(P, in_slot)), as_global<TOUT>(bslot(P, out_slot)),
        (const S *)P.s_inv[pass] + t, (const S *)P.s_ax[pass] + t, (const S *)P.s_ay[pass] + t,
        as_global<const int>(P.otab) + P.ooff[tb.tix], as_global<const S>(P.face[pass]) + P.foff[tb.tix],
        cs_from_prob ? P.c : 1.0, add_slot >= 0 ? as_global<const double>(bslot(P, add_slot)) : nullptr, 0.5 * P.c,
        smem);
}

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void __launch_bounds__(64) k_b_end_faces2d(const BTile *__restrict__ tiles, const BProb *__restrict__ probs, int sig0, int sig1,
                                                      int in_slot, int out_slot, int scale_by_piv) {
    extern __shared__ __align__(16) unsigned char smem[];
    const BTile tb = tiles[blockIdx.x >> 1];
    const BProb &P = probs[tb.prob];
    if (P.flags[0] == 0) return;
    const int sig[2] = {sig0, sig1};
    const EndFrame2 E = end_frame2(sig, P.n0, P.n1, tb.td);
    const GP<S> *dg[5] = {as_global<const S>(P.diagS[0]), as_global<const S>(P.diagS[1]),
                          as_global<const S>(P.diagS[2]), as_global<const S>(P.diagS[3]),
                          as_global<const S>(P.diagS[4])};
    if (blockIdx.x & 1)
        end_face2d_body<1, T, S, TIN, TOUT>(E, P.n0, dg, as_global<const S>(P.pivS),
                                            as_global<const TIN>(bslot(P, in_slot)), scale_by_piv != 0,
                                            as_global<TOUT>(bslot(P, out_slot)), smem);
    else
        end_face2d_body<0, T, S, TIN, TOUT>(E, P.n0, dg, as_global<const S>(P.pivS),
                                            as_global<const TIN>(bslot(P, in_slot)), scale_by_piv != 0,
                                            as_global<TOUT>(bslot(P, out_slot)), smem);
}

template <typename T, typename S, typename TIN, typename TOUT>
__global__ void k_b_end_corners2d(const BTile *__restrict__ tiles, int ntiles, const BProb *__restrict__ probs, int sig0, int sig1,
                                  int in_slot, int out_slot, int scale_by_piv) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntiles) return;
    const BTile tb = tiles[i];
    const BProb &P = probs[tb.prob];
    if (P.flags[0] == 0) return;
    const int sig[2] = {sig0, sig1};
    const EndFrame2 E = end_frame2(sig, P.n0, P.n1, tb.td);
    const GP<S> *dg[5] = {as_global<const S>(P.diagS[0]), as_global<const S>(P.diagS[1]),
                          as_global<const S>(P.diagS[2]), as_global<const S>(P.diagS[3]),
                          as_global<const S>(P.diagS[4])};
    end_corner2d_body<T, S, TIN, TOUT>(E, P.n0, dg, as_global<const S>(P.pivS), as_global<const TIN>(bslot(P, in_slot)),
                                       scale_by_piv != 0, as_global<TOUT>(bslot(P, out_slot)));
}

template <int R, typename T, typename S, typename TIN, typename TOUT>
static hipError_t b_fast_flags(const BTile *tiles, int ntiles, const BProb *probs, const int sig[2], int pass,
                               int in_slot, int out_slot, bool scale, bool coupled, bool csp, int add_slot, size_t lds,
                               hipStream_t st) {
    dim3 g(ntiles), b(256);
    const int c = csp ? 1 : 0;
    if (scale && coupled)
        hipLaunchKernelGGL((k_b_fast2d<R, T, S, TIN, TOUT, true, true>), g, b, lds, st, tiles, probs, sig[0], sig[1], pass, in_slot, out_slot, c, add_slot);
    else if (scale)
        hipLaunchKernelGGL((k_b_fast2d<R, T, S, TIN, TOUT, true, false>), g, b, lds, st, tiles, probs, sig[0], sig[1], pass, in_slot, out_slot, c, add_slot);
    else if (coupled)
        hipLaunchKernelGGL((k_b_fast2d<R, T, S, TIN, TOUT, false, true>), g, b, lds, st, tiles, probs, sig[0], sig[1], pass, in_slot, out_slot, c, add_slot);
    else
        hipLaunchKernelGGL((k_b_fast2d<R, T, S, TIN, TOUT, false, false>), g, b, lds, st, tiles, probs, sig[0], sig[1], pass, in_slot, out_slot, c, add_slot);
    return hipGetLastError();
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t b_fast_r(const BTile *tiles, int ntiles, const BProb *probs, const int sig[2], int pass, int R,
                           int in_slot, int out_slot, bool scale, bool coupled, bool csp, int add_slot, size_t lds,
                           hipStream_t st) {
    if (R == 1) return b_fast_flags<1, T, S, TIN, TOUT>(tiles, ntiles, probs, sig, pass, in_slot, out_slot, scale, coupled, csp, add_slot, lds, st);
    return b_fast_flags<2, T, S, TIN, TOUT>(tiles, ntiles, probs, sig, pass, in_slot, out_slot, scale, coupled, csp, add_slot, lds, st);
}

hipError_t launch_b_fast2d(const BTile *tiles, int ntiles, const BProb *probs, const int sig[2], int pass, int R,
                           Store s, int in_slot, bool in_f64, int out_slot, bool out_f64, bool scale, bool coupled,
                           bool csp, int add_slot, size_t lds, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
    if (add_slot >= 0 && !out_f64) return hipErrorInvalidValue;
#define PSW_B_ARGS tiles, ntiles, probs, sig, pass, R, in_slot, out_slot, scale, coupled, csp, add_slot, lds, st
    if (s == Store::F64) return b_fast_r<double, double, double, double>(PSW_B_ARGS);
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return b_fast_r<float, float, double, float>(PSW_B_ARGS);
        if (!in_f64 && out_f64) return b_fast_r<float, float, float, double>(PSW_B_ARGS);
        if (in_f64 && out_f64) return b_fast_r<float, float, double, double>(PSW_B_ARGS);
        return b_fast_r<float, float, float, float>(PSW_B_ARGS);
    }
    if (in_f64 && !out_f64) return b_fast_r<float, uint16_t, double, float>(PSW_B_ARGS);
    if (!in_f64 && out_f64) return b_fast_r<float, uint16_t, float, double>(PSW_B_ARGS);
    if (in_f64 && out_f64) return b_fast_r<float, uint16_t, double, double>(PSW_B_ARGS);
    return b_fast_r<float, uint16_t, float, float>(PSW_B_ARGS);
#undef PSW_B_ARGS
}

template <typename T, typename S, typename TIN, typename TOUT>
static hipError_t b_end_impl(const BTile *tiles, int ntiles, const BProb *probs, const int sig[2], int in_slot,
                             int out_slot, bool scale, int facemax, hipStream_t st) {
    size_t sm = sizeof(T) * 6 * ((size_t)facemax + 64); // chain data + scan area of 64 threads
    hipLaunchKernelGGL((k_b_end_faces2d<T, S, TIN, TOUT>), dim3(ntiles * 2), dim3(64), sm, st, tiles, probs, sig[0],
                       sig[1], in_slot, out_slot, scale ? 1 : 0);
    hipLaunchKernelGGL((k_b_end_corners2d<T, S, TIN, TOUT>), dim3((ntiles + 63) / 64), dim3(64), 0, st, tiles, ntiles,
                       probs, sig[0], sig[1], in_slot, out_slot, scale ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_b_end2d(const BTile *tiles, int ntiles, const BProb *probs, const int sig[2], Store s, int in_slot,
                          bool in_f64, int out_slot, bool out_f64, bool scale, int facemax, hipStream_t st) {
    if (ntiles <= 0) return hipSuccess;
#define PSW_E_ARGS tiles, ntiles, probs, sig, in_slot, out_slot, scale, facemax, st
    if (s == Store::F64) return b_end_impl<double, double, double, double>(PSW_E_ARGS);
    if (s == Store::F32) {
        if (in_f64 && !out_f64) return b_end_impl<float, float, double, float>(PSW_E_ARGS);
        if (!in_f64 && !out_f64) return b_end_impl<float, float, float, float>(PSW_E_ARGS);
        if (in_f64 && out_f64) return b_end_impl<float, float, double, double>(PSW_E_ARGS);
        return b_end_impl<float, float, float, double>(PSW_E_ARGS);
    }
    if (in_f64 && !out_f64) return b_end_impl<float, uint16_t, double, float>(PSW_E_ARGS);
    if (!in_f64 && !out_f64) return b_end_impl<float, uint16_t, float, float>(PSW_E_ARGS);
    if (in_f64 && out_f64) return b_end_impl<float, uint16_t, double, double>(PSW_E_ARGS);
    return b_end_impl<float, uint16_t, float, double>(PSW_E_ARGS);
#undef PSW_E_ARGS
}

} // namespace psw
