// psw_fast2d.h -- wavefront-pipelined 2D half-sweeps (see psw_fast2d.hip).
#pragma once

#include "psw_internal.h"

namespace psw {

// steps of coefficient loads each lane keeps in flight
constexpr int kFast2dDepth = 12;

struct Fast2dDiag {
    const double *d[5];
};

// One packed pass: geometry (direction of the pass), packed coefficients in
// the storage precision and per-tile offsets.
struct Fast2dPass {
    PassGeom g;
    int R;          // rows per lane (1 or 2)
    bool coupled;   // start faces coupled (false for the transposed passes)
    int lxmax, lymax;
    const void *s_inv, *s_ax, *s_ay, *face;
    const int64_t *toff, *foff;
};

size_t fast2d_lds_bytes(int lx, int ly, int R, size_t elem);

hipError_t launch_pack2d(const PassGeom &g, Store s, int R, bool transposed, const double *const *diag,
                         const double *piv, const int64_t *toff, const int64_t *foff, void *s_inv, void *s_ax,
                         void *s_ay, void *face, hipStream_t st);

hipError_t launch_fast2d(const Fast2dPass &p, Store s, const void *in, bool in_f64, bool scale_by_piv, void *out,
                         bool out_f64, double cscale, hipStream_t st);

hipError_t launch_end_faces2d_fast(const PassGeom &g, Store s, const void *const *diag, const void *piv,
                                   const void *in, bool in_f64, bool scale_by_piv, void *out, bool out_f64,
                                   int facemax, hipStream_t st);

// corners of an end-coupled pass only (psw_kernels.hip)
hipError_t launch_end_corners(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                              bool in_f64, bool scale_by_piv, void *out, bool out_f64, hipStream_t st);
// interior of an end-coupled pass only (psw_kernels.hip)
hipError_t launch_end_interior(const PassGeom &g, Store s, const void *const *diag, const void *piv, const void *in,
                               bool in_f64, bool scale_by_piv, void *out, bool out_f64, hipStream_t st);

} // namespace psw
