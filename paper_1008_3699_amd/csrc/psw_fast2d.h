// psw_fast2d.h -- wavefront-pipelined 2D half-sweeps (see psw_fast2d.hip).
#pragma once

#include "psw_internal.h"

namespace psw {

// Pipelined 2D passes.  The recurrence wave advances kFast2dBlk anti-diagonal
// steps between workgroup barriers; the other waves stage / write back one
// column block of kFast2dBlk columns per barrier interval.
constexpr int kFast2dBlk = 16;
// entries of a tile's step-offset table: [0] = bytes of the tile's packed
// region, [1 + t] = byte offset of step t's first lane slot minus the lane
// index times the slot size (so lane j reads at table value + j * slot).
inline int fast2d_tab_len(int lx, int ly, int R) { return 1 + lx + (ly + R - 1) / R - 1 + 3 * kFast2dBlk + 16; }
// packed elements of one tile: lx * L lane slots of R values, 64 zero slots, rounded to 256 bytes
inline int64_t fast2d_tile_elems(int lx, int ly, int R, size_t elem) {
    const int64_t L = (ly + R - 1) / R;
    const int64_t e = (int64_t)(lx * L + 64) * R;
    const int64_t a = (int64_t)(256 / elem);
    return (e + a - 1) / a * a;
}

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
    const int *otab;       // step-offset tables of all tiles
    const int64_t *ooff;   // per tile: start of its table in otab
};

size_t fast2d_lds_bytes(int lx, int ly, int R, size_t elem);

hipError_t launch_pack2d(const PassGeom &g, Store s, int R, bool transposed, const double *const *diag,
                         const double *piv, const int64_t *toff, const int64_t *foff, void *s_inv, void *s_ax,
                         void *s_ay, void *face, hipStream_t st);
// step-offset table of a tile (host); tab must hold fast2d_tab_len(lx, ly, R) entries
void fast2d_fill_tab(int lx, int ly, int R, size_t elem, int *tab);

// add (optional, FP64, requires out_f64): out = 0.5 * (cscale * result) + cadd * add
hipError_t launch_fast2d(const Fast2dPass &p, Store s, const void *in, bool in_f64, bool scale_by_piv, void *out,
                         bool out_f64, double cscale, const double *add, double cadd, hipStream_t st);

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

namespace psw {

// ---------------------------------------------------------------- batches
// A batch refers to problems that each own their buffers; device tables of
// pointers let one launch cover the tiles (or vector chunks) of all of them.
enum BSlot { kSlotR = 0, kSlotZ = 1, kSlotZ1 = 2, kSlotY1 = 3, kSlotY2 = 4, kSlotP = 5, kSlotQ = 6, kSlotX = 7,
             kSlotF = 8 };

struct BProb {
    int n0, n1;
    int64_t N;
    const void *s_inv[4], *s_ax[4], *s_ay[4], *face[4]; // packed passes (storage precision)
    const int64_t *toff, *foff;                         // per tile of this problem
    const int *otab;                                    // step-offset tables of this problem's tiles
    const int64_t *ooff;
    const void *diagS[5];                               // storage-precision couplings (end faces)
    const void *pivS;                                   // storage-precision pivots
    const double *diag64[5];                            // FP64 operator
    void *vec[9];                                       // r, z, z1, y1, y2, p, q, x, f
    double *scal;                                       // 0,1: r.z by parity; 2: p.q; 3: r.r; 4: f.f
    int *flags;                                         // 0: active, 1: iterations, 2: status
    double c;                                           // preconditioner scale
    int chunk0, nchunk;                                 // this problem's vector chunks
};

struct BTile {
    TileDesc td;
    int prob; // index into the problem table
    int tix;  // tile index within the problem
};

struct BChunk {
    int prob;
    int len;
    int64_t start;
};

// one pass of the preconditioner over all tiles in `tiles` (same R)
hipError_t launch_b_fast2d(const BTile *tiles, int ntiles, const BProb *probs, const int sig[2], int pass, int R,
                           Store s, int in_slot, bool in_f64, int out_slot, bool out_f64, bool scale_by_piv,
                           bool coupled, bool cs_from_prob, int add_slot, size_t lds, hipStream_t st);
// end faces and cross points of an end-coupled pass over all tiles
hipError_t launch_b_end2d(const BTile *tiles, int ntiles, const BProb *probs, const int sig[2], Store s, int in_slot,
                          bool in_f64, int out_slot, bool out_f64, bool scale_by_piv, int facemax, hipStream_t st);

} // namespace psw
