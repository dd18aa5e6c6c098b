// psw_internal.h -- types shared by the HIP kernels and the host runtime of
// libpsweep.so.  Not part of the public ABI (include/psweep.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psw {

// One subdomain (a "tile"): lower corner, extent and coordinate parity per
// axis.  Unused axes have lo = 0, len = 1, par = 0.
struct TileDesc {
    int lo[3];
    int len[3];
    int par[3];
};

// Storage precisions of the diagonals used by the preconditioner sweeps.
enum class Store { F64 = 0, F32 = 1, BF16 = 2 };

// The one FP64 -> BF16 conversion of the library: round to nearest, ties to
// even.  The value is first rounded to FP32 by truncation with a sticky bit
// (round to odd), which keeps every bit below the BF16 rounding position that
// decides the rounding, then rounded to nearest even at bit 16.  Used for the
// stored coefficients of every BF16 path.
__device__ __forceinline__ uint16_t f64_to_bf16(double x) {
    const float t = __double2float_rz(x);
    uint32_t u = __float_as_uint(t);
    if ((double)t != x && (u & 0x7f800000u) != 0x7f800000u) u |= 1u;
    const uint32_t r = u + 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(r >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }

// Geometry of one sweep pass: grid, tile table and the base direction of the
// pass (the direction of tile (0,0,0); the sign on axis a flips for odd tile
// coordinate a, so neighbouring tiles sweep in opposite directions).
struct PassGeom {
    int dim;
    int n[3];
    int sig[3];
    int ntiles;
    const TileDesc *tiles;
    int cmax;  // largest tile cross-section (len1*len2)
    int l1max; // largest len1
    int l2max; // largest len2
};

// Kernel launchers (defined in psw_kernels.hip).  Every launcher returns a
// hipError_t and launches on `st`.

// Stationary decomposed SOR sweep, FP64 (start-coupled, per-corner omega).
hipError_t launch_sweep_stationary(const PassGeom &g, const double *const *diag, const double *omega8,
                                   const double *uold, const double *f, double *out, hipStream_t st);

// Restricted-overlap sweep (one workgroup per subdomain, widened box and a ring in LDS).
// ras_lds_bytes: LDS bytes for the largest subdomain, 0 if it does not fit lds_limit.
size_t ras_lds_bytes(const PassGeom &g, const int lenmax[3], int overlap, size_t lds_limit);
hipError_t launch_ras(const PassGeom &g, const double *const *diag, const double *omega8, int overlap, size_t lds,
                      const double *uold, const double *f, double *out, hipStream_t st);

// Stationary sweep as a start-coupled pass (2D): right-hand side f + (1/w - 1) a^P u_old + N2 u_old
// and pivots a^P / w, with w per point from its subdomain's start corner under the direction map sig
// (omega8: the 4 factors by start corner, host array, passed by value).
hipError_t launch_sor_rhs2d(const int n[3], const int p[3], const int sig[3], const double *const *diag,
                           const double *omega8, const double *f, const double *uold, double *out, hipStream_t st);
hipError_t launch_sor_piv2d(const int n[3], const int p[3], const int sig[3], const double *aP, const double *omega8,
                            double *piv, hipStream_t st);

// Preconditioner half-sweep, start-coupled: out = cscale * (Piv - N)^-1 (in .* (scale_by_piv ? Piv : 1)).
// in/out element types follow `in_f64`/`out_f64`; arithmetic in FP64 for Store::F64, else FP32.
hipError_t launch_half_start(const PassGeom &g, Store s, const void *const *diag, const void *piv,
                             const void *in, bool in_f64, bool scale_by_piv, void *out, bool out_f64,
                             double cscale, hipStream_t st);

// Transposed half-sweep, end-coupled: interior phase, then the coupled end
// faces (2D: face chains then cross points; 3D: faces, edges, corners).
// out = (Piv - N)^-T (in .* (scale_by_piv ? Piv : 1)) where N are the upstream
// couplings of the direction map -sig (the solve itself runs along sig).
hipError_t launch_half_end(const PassGeom &g, Store s, const void *const *diag, const void *piv,
                           const void *in, bool in_f64, bool scale_by_piv, void *out, bool out_f64,
                           hipStream_t st);

// 3D half-sweeps with the whole tile in LDS (FP32 arithmetic; FP32 or BF16 storage).
// Packed coefficients per pass: pack3_slot_bytes(s) per slot, level-major per tile,
// (len0 + len1 + len2 - 2) * len1 * len2 slots from poff[tile].
size_t pack3_slot_bytes(Store s);
size_t tile3_lds_bytes(const PassGeom &g, int len0max, size_t elem);
hipError_t launch_pack3(const PassGeom &g, Store s, bool transposed, const double *const *diag, const double *piv,
                        const int64_t *poff, void *pk, hipStream_t st);
// start: the start-coupled pass (out = cscale * result); else the interior of an
// end-coupled pass, to be followed by launch_end_fixups3
hipError_t launch_tile3(const PassGeom &g, Store s, bool start, const void *const *diag, const void *piv,
                        const void *pk, const int64_t *poff, int len0max, const void *in, bool in_f64,
                        bool scale_by_piv, void *out, bool out_f64, double cscale, void *fimg, hipStream_t st);
// Coefficient image of the coupled start faces of a start-coupled pass (fimg above, or null):
// its size in FP32 elements (0 if the face kernel with gathered records does not apply), and
// the kernel that writes it from the pass's diagonals and pivots.
int64_t faces3_image_elems(const PassGeom &g, int len0max, size_t lds_limit);
hipError_t launch_faces3_image(const PassGeom &g, Store s, const void *const *diag, const void *piv, int len0max,
                               size_t lds_limit, void *img, hipStream_t st);
hipError_t launch_end_fixups3(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                              bool in_f64, bool scale_by_piv, void *out, bool out_f64, int len0max, void *eimg,
                              hipStream_t st);
// Coefficient image of the coupled end faces of an end-coupled pass (eimg above, or null).
int64_t end_faces3_image_elems(const PassGeom &g, int len0max, size_t lds_limit);
hipError_t launch_end_faces3_image(const PassGeom &g, Store s, const void *const *diag, const void *piv, int len0max,
                                   size_t lds_limit, void *img, hipStream_t st);

// ILU(0) pivots of the decomposed factorisation, FP64.
hipError_t launch_ilu_pivots(const PassGeom &g, const double *const *diag, double *piv, int *bad,
                             hipStream_t st);

// Vector kernels (FP64, natural layout).
hipError_t launch_assemble(int dim, const int n[3], const double *const *alpha, double beta,
                           double *const *diag, hipStream_t st);
hipError_t launch_spmv(int dim, const int n[3], const double *const *diag, const double *x, double *y,
                       hipStream_t st);
// the same with the lower couplings read as the neighbours' upper ones (symmetric storage only)
hipError_t launch_spmv_sym(int dim, const int n[3], const double *const *diag, const double *x, double *y,
                           hipStream_t st);
// 3D q = A x marching through z runs; sym: the lower couplings read as the neighbours' upper ones
hipError_t launch_spmv3(const int n[3], const double *const *diag, bool sym, const double *x, double *q,
                        hipStream_t st);
// flag[0] (set to 1 by the caller) becomes 0 unless every lower coupling equals the neighbour's upper one
hipError_t launch_sym_check(int dim, const int n[3], const double *const *diag, int *flag, hipStream_t st);
hipError_t launch_convert(const double *src, void *dst, Store s, int64_t N, double scale, hipStream_t st);
hipError_t launch_scale_add(double *z, const double *a, double ca, const void *b, bool b_f64, double cb,
                            int64_t N, hipStream_t st);

// Deterministic reductions: partial sums per block in fixed order, then one
// block sums the partials in fixed order.  `partials` holds kRedBlocks doubles.
constexpr int kRedBlocks = 1024;
// most blocks (and p.q partials) of the fused 3D CG step
constexpr int kCgPq3dMaxBlocks = 2 * kRedBlocks;
constexpr int kRedThreads = 256;
hipError_t launch_dot(const double *x, const double *y, int64_t N, double *partials, double *out,
                      hipStream_t st);

// CG helpers with device-resident scalars.
// per-block partial sums of x.y (kRedBlocks of them)
hipError_t launch_dot_partial(const double *x, const double *y, int64_t N, double *partials, hipStream_t st);
// r.z partials with z = 0.5 z1 + b z2 formed on the fly (z2 in FP64, or in FP32: the output of
// FP32/BF16 sweeps)
hipError_t launch_dot_partial_zz(const double *r, const double *z1, const double *z2, double b, int64_t N,
                                 double *partials, hipStream_t st);
hipError_t launch_dot_partial_zf(const double *r, const double *z1, const float *z2, double b, int64_t N,
                                 double *partials, hipStream_t st);
// y += a[0] x, a on the device
hipError_t launch_axpy_dev(double *y, const double *a, const double *x, int64_t N, hipStream_t st);
// Fused CG step on a 2D grid (5-point operator in diag[0..4]): beta = rz / rz_old[0] with rz the
// sum of kRedBlocks partials (stored to rz_new[0]; beta = 0 when first), pnew = z + beta pold,
// x += alpha_prev[0] pold (skipped when first), q = A pnew, and *npq (<= kRedBlocks) partials of p.q.
// z = 0.5 z1 + hb z2 when z2 is given, else z1.  pnew must not alias pold.
hipError_t launch_cg_pq2d(int n0, int n1, const double *const *diag, const double *z1, const double *z2, double hb,
                          const double *pold, double *pnew, double *q, double *x, const double *rz_part,
                          double *rz_new, const double *rz_old, const double *alpha_prev, bool first,
                          double *pq_part, int *npq, bool sym, hipStream_t st);
// The same on a 3D grid (7-point operator in diag[0..6]); z = 0.5 z1 + hb z2 with z2 in FP32 when
// given, else z1.  pnew must not alias pold.  *npq <= kCgPq3dMaxBlocks partials of p.q.
hipError_t launch_cg_pq3d(const int n[3], const double *const *diag, const double *z1, const float *z2, double hb,
                          const double *pold, double *pnew, double *q, double *x, const double *rz_part,
                          double *rz_new, const double *rz_old, const double *alpha_prev, bool first,
                          double *pq_part, int *npq, bool sym, hipStream_t st);
// r -= alpha q, alpha = rz[0] / (sum of npq partials); out[0] = p.q, out[1] = alpha,
// out[2 .. 2 + kRedBlocks) = partials of r.r; the same to hout (device-visible pinned host memory) if given
hipError_t launch_cg_r(double *r, const double *q, const double *rz, const double *pq_part, int npq, double *out,
                       int64_t N, double *hout, hipStream_t st);
hipError_t launch_copy_scaled(double *y, const double *x, double a, int64_t N, hipStream_t st);
hipError_t launch_residual(int dim, const int n[3], const double *const *diag, const double *f,
                           const double *x, double *r, hipStream_t st);
// GMRES: y = sum_j c[j] * V[j] (c on device), V rows of length N.
hipError_t launch_multi_axpy(double *y, const double *V, const double *c, int k, int64_t N, bool accumulate,
                             hipStream_t st);
// GMRES: out[j] = V[j] . w for j < k (deterministic), using partials of k*kRedBlocks.
hipError_t launch_multi_dot(const double *V, const double *w, int k, int64_t N, double *partials, double *out,
                            hipStream_t st);

} // namespace psw
