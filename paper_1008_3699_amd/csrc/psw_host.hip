// psw_host.hip -- host runtime and C ABI of libpsweep.so (see include/psweep.h).
//
// A psw_problem owns FP64 device copies of the diagonals, the subdomain
// ("tile") table, the preconditioner state (pivots and diagonals in the sweep
// precision) and the Krylov workspace.  Every kernel runs on the caller's
// stream; scalars of the Krylov recurrences stay on the device and only the
// residual norm crosses to the host for the stopping test.
#include "psw_internal.h"
#include "psw_fast2d.h"
#include "psw_batch.h"
#include "../../include/psweep.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <tuple>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

using namespace psw;

namespace {

// Base direction cycle of tile (0,0,0) (Sec. 3, Sweeping directions; Sec. 4 for 3D):
// consecutive pairs are mutually reversed and each pair uses a new diagonal.
const int kCycle1[2][3] = {{+1, 1, 1}, {-1, 1, 1}};
const int kCycle2[4][3] = {{-1, -1, 1}, {+1, +1, 1}, {+1, -1, 1}, {-1, +1, 1}};
const int kCycle3[8][3] = {{-1, -1, -1}, {+1, +1, +1}, {+1, -1, -1}, {-1, +1, +1},
                           {-1, +1, -1}, {+1, -1, +1}, {+1, +1, -1}, {-1, -1, +1}};

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    ~DevBuf() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    bool ensure(size_t b) {
        if (bytes >= b && p) return true;
        release();
        if (hipMalloc(&p, b) != hipSuccess) {
            p = nullptr;
            return false;
        }
        bytes = b;
        return true;
    }
    template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

size_t store_bytes(Store s) { return s == Store::F64 ? 8 : (s == Store::F32 ? 4 : 2); }

} // namespace

struct FastPassBuf {
    DevBuf inv, ax, ay, face;
};

// A second stream and two events: work that does not depend on the main
// stream's next kernels forks onto it and joins back (also under capture).
struct SideStream {
    hipStream_t s = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
    ~SideStream() {
        if (fork) (void)hipEventDestroy(fork);
        if (join) (void)hipEventDestroy(join);
        if (s) (void)hipStreamDestroy(s);
    }
    bool ensure() {
        if (s) return true;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) return false;
        if (hipEventCreateWithFlags(&fork, hipEventDisableTiming) != hipSuccess) return false;
        if (hipEventCreateWithFlags(&join, hipEventDisableTiming) != hipSuccess) return false;
        return true;
    }
};

// pinned host scalars and an event, for reading a device result without draining the stream
struct HostScalars {
    double *p = nullptr;
    hipEvent_t ev = nullptr;
    ~HostScalars() {
        if (ev) (void)hipEventDestroy(ev);
        if (p) (void)hipHostFree(p);
    }
    bool ensure() {
        if (p) return true;
        if (hipHostMalloc((void **)&p, (8 + kRedBlocks) * sizeof(double), hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            return false;
        }
        return hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
    }
};

// timing of one pipelined pass inside solves: events around every kStride-th launch
struct PassTiming {
    static constexpr int kPool = 1024, kStride = 8;
    bool on = false;
    int which = 0;
    int64_t calls = 0, used = 0;
    std::vector<hipEvent_t> ev; // 2 * kPool
    ~PassTiming() {
        for (hipEvent_t e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

struct PrecState {
    bool ready = false;
    double omega = 1.0;
    double c = 1.0;
    DevBuf diag[7]; // off-diagonals in sweep precision (index 0 unused)
    DevBuf piv;     // pivots in sweep precision
    DevBuf piv64;   // pivots in FP64
    // pipelined 2D path: packed coefficients of the four passes
    bool fast = false;
    int R = 1, lxmax = 1, lymax = 1;
    FastPassBuf fp[4];
    DevBuf toff, foff; // per tile: start of its packed coefficients / face records
    DevBuf otab, ooff; // step-offset tables and their per-tile starts
    // 3D path with the tile in LDS (FP32 arithmetic): level-major packed coefficients
    bool tile3 = false;
    int len0max = 1;
    DevBuf t3pk[4], t3off;
    DevBuf f3img[2];        // coefficient images of the coupled start faces, passes 0 and 1
    bool f3ok[2] = {false, false};
    DevBuf e3img[2];        // coefficient images of the coupled end faces, passes 2 and 3
    bool e3ok[2] = {false, false};
};

// The stationary sweep on the pipelined 2D passes (2D problems, and 1D ones as n x 1 grids): the
// direction maps of the schedule cycle (index c of the base cycle) packed as start-coupled passes
// with pivots a^P / w.
struct StatState {
    bool ready = false;
    bool fast = false;
    int R = 1, lxmax = 1, lymax = 1;
    FastPassBuf fp[4];
    DevBuf toff, foff, otab, ooff;
};

struct psw_problem {
    int device = 0;
    int dim = 2; // the problem's dimension (ABI)
    int kd = 2;  // dimension the kernels see: a 1D problem runs as an n x 1 grid (zero S/N couplings)
    int n[3] = {1, 1, 1};
    int64_t N = 0;
    bool has_diag = false;
    // the FP64 diagonals store a symmetric operator (a^W(P) = a^E(P - e_x), ...), bit for bit:
    // checked once per set of diagonals; the Krylov loops' SpMV then reads the upper couplings only
    bool sym = false;
    DevBuf symflag;
    psw_prec prec = PSW_F64;
    DevBuf diag[7];
    double omega[8] = {1, 1, 1, 1, 1, 1, 1, 1};
    int p[3] = {1, 1, 1};
    int overlap = 2;
    int phase = 0;
    bool has_decomp = false;
    bool force_generic = false; // psw_set_path(PSW_PATH_GENERIC): level kernels for every pass
    DevBuf tiles;
    int ntiles = 0;
    int cmax = 1, l1max = 1, l2max = 1;
    PrecState pc[2];
    StatState stat;
    // workspace
    DevBuf w_r, w_z, w_p, w_q, w_t, w_y, w_y2, w_z1;
    DevBuf w_y3; // the transposed chain's output in sweep precision (3D LDS-tile passes)
    DevBuf partials, scal;
    DevBuf gm_V, gm_Z, gm_h;
    size_t lds_limit = 65536;
    SideStream side;
    HostScalars hs;
    PassTiming timing[5]; // per pass 0..3, and 4: the fused 2D CG step
    int timing_last = 0;
};

static hipError_t krylov_spmv(psw_problem *P, const double *const *d, const double *p, double *q, hipStream_t st);

namespace {

#define HIPCHK(x)                                                                                                  \
    do {                                                                                                           \
        hipError_t e_ = (x);                                                                                       \
        if (e_ != hipSuccess) {                                                                                    \
            return PSW_EDEVICE;                                                                                    \
        }                                                                                                          \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
        else prev = -1;
        (void)hipGetLastError(); // drop an error left by an earlier, already reported call
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

void partition(int n, int p, std::vector<int> &lo, std::vector<int> &len) {
    lo.resize(p);
    len.resize(p);
    int base = n / p, rem = n % p, s = 0;
    for (int r = 0; r < p; ++r) {
        len[r] = base + (r < rem ? 1 : 0);
        lo[r] = s;
        s += len[r];
    }
}

PassGeom geom(const psw_problem *P, const int sig[3]) {
    PassGeom g{};
    g.dim = P->kd;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = P->n[a];
        g.sig[a] = a < P->kd ? sig[a] : 1;
    }
    g.ntiles = P->ntiles;
    g.tiles = P->tiles.as<TileDesc>();
    g.cmax = P->cmax;
    g.l1max = P->l1max;
    g.l2max = P->l2max;
    return g;
}

// entry c of the base direction cycle of the problem's dimension
void cycle_sig(const psw_problem *P, int c, int sig[3]) {
    const int *s = P->dim == 1 ? kCycle1[c] : P->dim == 2 ? kCycle2[c] : kCycle3[c];
    for (int a = 0; a < 3; ++a) sig[a] = a < P->dim ? s[a] : 1;
}

// cycle entry of schedule step it (phase swaps the members of every pair)
int sched_step(const psw_problem *P, int64_t it) {
    int k = (int)(it % (1 << P->dim));
    return P->phase ? k ^ 1 : k;
}

void sched_sig(const psw_problem *P, int64_t it, int sig[3]) { cycle_sig(P, sched_step(P, it), sig); }

Store store_of(psw_prec p) { return p == PSW_F64 ? Store::F64 : (p == PSW_F32 ? Store::F32 : Store::BF16); }

const double *const *diag64(const psw_problem *P, const double **tmp) {
    for (int k = 0; k < 7; ++k) tmp[k] = P->diag[k].as<const double>();
    return tmp;
}

psw_status ensure_work(psw_problem *P) {
    size_t b = sizeof(double) * (size_t)P->N;
    if (!P->w_r.ensure(b) || !P->w_z.ensure(b) || !P->w_p.ensure(b) || !P->w_q.ensure(b) || !P->w_t.ensure(b) ||
        !P->w_y.ensure(b) || !P->w_y2.ensure(b) || !P->w_z1.ensure(b) ||
        !P->partials.ensure(sizeof(double) * kRedBlocks * 64) || !P->scal.ensure(sizeof(double) * 64))
        return PSW_ENOMEM;
    return PSW_OK;
}

psw_status check_lds(const psw_problem *P, size_t elem) {
    size_t need = elem * (size_t)(4 * P->cmax + 4 * P->l2max + 4 * P->l1max + 2);
    return need <= P->lds_limit ? PSW_OK : PSW_ENOTSUP;
}

// direction of pass `which` (0: d, 1: -d, 2: d transposed, 3: -d transposed)
void pass_sig(const psw_problem *P, int which, int sig[3]) {
    sched_sig(P, 0, sig);
    if (which == 1 || which == 3)
        for (int a = 0; a < 3; ++a) sig[a] = -sig[a];
}

// whether a 2D decomposition runs on the pipelined passes, with rows per lane and largest tile
bool fast_shape(int dim, const int n[3], const int p[3], psw_prec prec, size_t lds_limit, int &R, int &lxmax,
                int &lymax) {
    if (dim != 2) return false;
    std::vector<int> lo, len;
    partition(n[0], p[0], lo, len);
    lxmax = *std::max_element(len.begin(), len.end());
    partition(n[1], p[1], lo, len);
    lymax = *std::max_element(len.begin(), len.end());
    R = (lymax + 63) / 64;
    if (R > 2) return false;
    size_t elem = prec == PSW_F64 ? 8 : 4;
    return fast2d_lds_bytes(lxmax, lymax, R, elem) <= lds_limit;
}

bool fast_eligible(const psw_problem *P, int &R, int &lxmax, int &lymax) {
    if (P->force_generic) return false;
    return fast_shape(P->kd, P->n, P->p, P->prec, P->lds_limit, R, lxmax, lymax);
}

// Sizes of the pipelined 2D packing: elements of one pass's packed coefficients (t) and face
// records (f, before the 8 spare slots), and entries of the step-offset tables (otab); the
// formulas fast_setup allocates with.
struct Fast2dPlan {
    int64_t t = 0, f = 0, otab = 0;
};
Fast2dPlan fast2d_plan(const int n[3], const int p[3], int R, size_t eb) {
    std::vector<int> lo0, len0, lo1, len1;
    partition(n[0], p[0], lo0, len0);
    partition(n[1], p[1], lo1, len1);
    Fast2dPlan pl;
    for (int s1 = 0; s1 < p[1]; ++s1)
        for (int s0 = 0; s0 < p[0]; ++s0) {
            const int lx = len0[s0], ly = len1[s1];
            pl.t += fast2d_tile_elems(lx, ly, R, eb);
            pl.f += 4 * (int64_t)(lx + ly) + 3;
            pl.f = (pl.f + 7) & ~(int64_t)7;
            pl.otab += fast2d_tab_len(lx, ly, R);
        }
    return pl;
}

// slots of one 3D LDS-tile pass's level-major packing (tile3_setup)
int64_t tile3_slots(const int n[3], const int p[3]) {
    std::vector<int> lo[3], len[3];
    for (int a = 0; a < 3; ++a) partition(n[a], p[a], lo[a], len[a]);
    int64_t tot = 0;
    for (int t = 0; t < p[2]; ++t)
        for (int u = 0; u < p[1]; ++u)
            for (int r = 0; r < p[0]; ++r)
                tot += (int64_t)(len[0][r] + len[1][u] + len[2][t] - 2) * len[1][u] * len[2][t];
    return tot;
}

psw_status fast_setup(psw_problem *P, PrecState &S, hipStream_t st) {
    int R, lxmax, lymax;
    S.fast = false;
    if (!fast_eligible(P, R, lxmax, lymax)) return PSW_OK;
    std::vector<int> lo0, len0, lo1, len1;
    partition(P->n[0], P->p[0], lo0, len0);
    partition(P->n[1], P->p[1], lo1, len1);
    Store s = store_of(P->prec);
    size_t eb = store_bytes(s);
    std::vector<int64_t> toff, foff, ooff;
    std::vector<int> otab;
    int64_t t = 0, f = 0;
    for (int s1 = 0; s1 < P->p[1]; ++s1)
        for (int s0 = 0; s0 < P->p[0]; ++s0) {
            const int lx = len0[s0], ly = len1[s1];
            toff.push_back(t);
            foff.push_back(f);
            ooff.push_back((int64_t)otab.size());
            t += fast2d_tile_elems(lx, ly, R, eb);
            f += 4 * (int64_t)(lx + ly) + 3;
            f = (f + 7) & ~(int64_t)7;
            const size_t o = otab.size();
            otab.resize(o + fast2d_tab_len(lx, ly, R));
            fast2d_fill_tab(lx, ly, R, eb, otab.data() + o);
        }
    if (!S.toff.ensure(sizeof(int64_t) * toff.size()) || !S.foff.ensure(sizeof(int64_t) * foff.size()) ||
        !S.ooff.ensure(sizeof(int64_t) * ooff.size()) || !S.otab.ensure(sizeof(int) * otab.size()))
        return PSW_ENOMEM;
    HIPCHK(hipMemcpy(S.toff.p, toff.data(), sizeof(int64_t) * toff.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.foff.p, foff.data(), sizeof(int64_t) * foff.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.ooff.p, ooff.data(), sizeof(int64_t) * ooff.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.otab.p, otab.data(), sizeof(int) * otab.size(), hipMemcpyHostToDevice));
    const double *d[7];
    diag64(P, d);
    for (int w = 0; w < 4; ++w) {
        FastPassBuf &B = S.fp[w];
        if (!B.inv.ensure(eb * t) || !B.ax.ensure(eb * t) || !B.ay.ensure(eb * t) || !B.face.ensure(eb * (f + 8)))
            return PSW_ENOMEM;
        int sig[3];
        pass_sig(P, w, sig);
        PassGeom g = geom(P, sig);
        HIPCHK(launch_pack2d(g, s, R, w >= 2, d, S.piv64.as<double>(), S.toff.as<int64_t>(), S.foff.as<int64_t>(),
                             B.inv.p, B.ax.p, B.ay.p, B.face.p, st));
    }
    S.R = R;
    S.lxmax = lxmax;
    S.lymax = lymax;
    S.fast = true;
    return PSW_OK;
}

// Stationary sweep state: step-offset tables as fast_setup, and per direction map of the cycle the
// pivots a^P / w (w by each subdomain's start corner) packed with the upstream couplings.
psw_status stat_setup(psw_problem *P, hipStream_t st) {
    StatState &S = P->stat;
    S.fast = false;
    S.ready = true;
    int R, lxmax, lymax;
    if (P->kd != 2 || P->force_generic || !fast_shape(2, P->n, P->p, PSW_F64, P->lds_limit, R, lxmax, lymax))
        return PSW_OK;
    std::vector<int> lo0, len0, lo1, len1;
    partition(P->n[0], P->p[0], lo0, len0);
    partition(P->n[1], P->p[1], lo1, len1);
    const size_t eb = 8;
    std::vector<int64_t> toff, foff, ooff;
    std::vector<int> otab;
    int64_t t = 0, f = 0;
    for (int s1 = 0; s1 < P->p[1]; ++s1)
        for (int s0 = 0; s0 < P->p[0]; ++s0) {
            const int lx = len0[s0], ly = len1[s1];
            toff.push_back(t);
            foff.push_back(f);
            ooff.push_back((int64_t)otab.size());
            t += fast2d_tile_elems(lx, ly, R, eb);
            f += 4 * (int64_t)(lx + ly) + 3;
            f = (f + 7) & ~(int64_t)7;
            const size_t o = otab.size();
            otab.resize(o + fast2d_tab_len(lx, ly, R));
            fast2d_fill_tab(lx, ly, R, eb, otab.data() + o);
        }
    S.ready = false;
    if (!S.toff.ensure(sizeof(int64_t) * toff.size()) || !S.foff.ensure(sizeof(int64_t) * foff.size()) ||
        !S.ooff.ensure(sizeof(int64_t) * ooff.size()) || !S.otab.ensure(sizeof(int) * otab.size()))
        return PSW_ENOMEM;
    HIPCHK(hipMemcpy(S.toff.p, toff.data(), sizeof(int64_t) * toff.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.foff.p, foff.data(), sizeof(int64_t) * foff.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.ooff.p, ooff.data(), sizeof(int64_t) * ooff.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(S.otab.p, otab.data(), sizeof(int) * otab.size(), hipMemcpyHostToDevice));
    psw_status ps = ensure_work(P);
    if (ps) return ps;
    double *piv = P->w_y.as<double>(); // pivots of one direction map at a time, consumed by the packing
    const double *d[7];
    diag64(P, d);
    for (int c = 0; c < (1 << P->dim); ++c) {
        FastPassBuf &B = S.fp[c];
        if (!B.inv.ensure(eb * t) || !B.ax.ensure(eb * t) || !B.ay.ensure(eb * t) || !B.face.ensure(eb * (f + 8)))
            return PSW_ENOMEM;
        int sig[3];
        cycle_sig(P, c, sig);
        HIPCHK(launch_sor_piv2d(P->n, P->p, sig, d[0], P->omega, piv, st));
        const PassGeom g = geom(P, sig);
        HIPCHK(launch_pack2d(g, Store::F64, R, false, d, piv, S.toff.as<int64_t>(), S.foff.as<int64_t>(), B.inv.p,
                             B.ax.p, B.ay.p, B.face.p, st));
    }
    S.R = R;
    S.lxmax = lxmax;
    S.lymax = lymax;
    S.fast = true;
    S.ready = true;
    return PSW_OK;
}

// 3D problems swept in FP32 whose tiles fit in LDS: pack the four passes' coefficients
psw_status tile3_setup(psw_problem *P, PrecState &S, hipStream_t st) {
    S.tile3 = false;
    S.f3ok[0] = S.f3ok[1] = false;
    S.e3ok[0] = S.e3ok[1] = false;
    if (P->dim != 3 || P->prec == PSW_F64 || P->cmax > 1024 || P->force_generic) return PSW_OK;
    std::vector<int> lo[3], len[3];
    for (int a = 0; a < 3; ++a) partition(P->n[a], P->p[a], lo[a], len[a]);
    const int len0max = *std::max_element(len[0].begin(), len[0].end());
    int sig[3];
    pass_sig(P, 0, sig);
    if (tile3_lds_bytes(geom(P, sig), len0max, sizeof(float)) > P->lds_limit) return PSW_OK;
    // slots per tile, in the tile order of the decomposition (x fastest)
    std::vector<int64_t> off;
    int64_t tot = 0;
    for (int t = 0; t < P->p[2]; ++t)
        for (int u = 0; u < P->p[1]; ++u)
            for (int r = 0; r < P->p[0]; ++r) {
                off.push_back(tot);
                const int64_t C = (int64_t)len[1][u] * len[2][t];
                tot += (int64_t)(len[0][r] + len[1][u] + len[2][t] - 2) * C;
            }
    if ((int)off.size() != P->ntiles) return PSW_EINVAL;
    const Store s = store_of(P->prec);
    if (!S.t3off.ensure(sizeof(int64_t) * off.size())) return PSW_ENOMEM;
    HIPCHK(hipMemcpy(S.t3off.p, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice));
    const double *d[7];
    diag64(P, d);
    for (int w = 0; w < 4; ++w) {
        if (!S.t3pk[w].ensure(pack3_slot_bytes(s) * (size_t)tot)) return PSW_ENOMEM;
        pass_sig(P, w, sig);
        HIPCHK(launch_pack3(geom(P, sig), s, w >= 2, d, S.piv64.as<double>(), S.t3off.as<int64_t>(), S.t3pk[w].p,
                            st));
    }
    // coefficient images of the coupled faces, from the sweep-precision diagonals and pivots:
    // the start faces of passes 0 and 1, the end faces of passes 2 and 3 (none where the face
    // kernels with gathered records do not apply; those passes gather everything)
    const void *ds[7];
    for (int k = 0; k < 7; ++k) ds[k] = S.diag[k].p;
    for (int w = 0; w < 4; ++w) {
        pass_sig(P, w, sig);
        const PassGeom g = geom(P, sig);
        const int e = w & 1;
        DevBuf &img = w <= 1 ? S.f3img[e] : S.e3img[e];
        bool &ok = w <= 1 ? S.f3ok[e] : S.e3ok[e];
        const int64_t ne = w <= 1 ? faces3_image_elems(g, len0max, P->lds_limit)
                                  : end_faces3_image_elems(g, len0max, P->lds_limit);
        if (ne <= 0) continue;
        if (!img.ensure(sizeof(float) * (size_t)ne)) return PSW_ENOMEM;
        if (w <= 1)
            HIPCHK(launch_faces3_image(g, s, ds, S.piv.p, len0max, P->lds_limit, img.p, st));
        else
            HIPCHK(launch_end_faces3_image(g, s, ds, S.piv.p, len0max, P->lds_limit, img.p, st));
        ok = true;
    }
    S.len0max = len0max;
    S.tile3 = true;
    return PSW_OK;
}

// preconditioner state for kind (SSOR: Piv = D/w, c = 2-w; ILU0: Piv = D~, c = 1)
psw_status precond_setup(psw_problem *P, psw_precond kind, hipStream_t st) {
    if (kind != PSW_SSOR && kind != PSW_ILU0) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    PrecState &S = P->pc[kind];
    if (S.ready) return PSW_OK;
    Store s = store_of(P->prec);
    psw_status ps = check_lds(P, 8);
    if (ps) return ps;
    if ((ps = ensure_work(P))) return ps;
    size_t eb = store_bytes(s) * (size_t)P->N;
    for (int k = 1; k < 2 * P->kd + 1; ++k) {
        if (!S.diag[k].ensure(eb)) return PSW_ENOMEM;
        HIPCHK(launch_convert(P->diag[k].as<double>(), S.diag[k].p, s, P->N, 1.0, st));
    }
    if (!S.piv.ensure(eb) || !S.piv64.ensure(sizeof(double) * (size_t)P->N)) return PSW_ENOMEM;
    if (kind == PSW_SSOR) {
        S.omega = P->omega[0];
        S.c = 2.0 - S.omega;
        HIPCHK(launch_copy_scaled(S.piv64.as<double>(), P->diag[0].as<double>(), 1.0 / S.omega, P->N, st));
    } else {
        S.c = 1.0;
        int sig[3];
        sched_sig(P, 0, sig);
        PassGeom g = geom(P, sig);
        const double *d[7];
        int *bad = reinterpret_cast<int *>(P->scal.as<double>() + 63);
        HIPCHK(hipMemsetAsync(bad, 0, sizeof(int), st));
        HIPCHK(launch_ilu_pivots(g, diag64(P, d), S.piv64.as<double>(), bad, st));
        int hb = 0;
        HIPCHK(hipMemcpyAsync(&hb, bad, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPCHK(hipStreamSynchronize(st));
        if (hb) return PSW_EPIVOT;
    }
    HIPCHK(launch_convert(S.piv64.as<double>(), S.piv.p, s, P->N, 1.0, st));
    if ((ps = fast_setup(P, S, st))) return ps;
    if ((ps = tile3_setup(P, S, st))) return ps;
    S.ready = true;
    return PSW_OK;
}

// Device bytes that a problem holds after a CG solve with preconditioner kind (diagonals,
// tile table, workspace, the preconditioner's sweep-precision state and packings, the 3D
// transposed chain's buffer), from the size formulas its set-up allocates with.
size_t problem_bytes(int dim, const int n_in[3], const int p_in[3], psw_prec prec, psw_precond kind,
                     size_t lds_limit) {
    int n[3] = {1, 1, 1}, p[3] = {1, 1, 1};
    int64_t N = 1;
    for (int a = 0; a < dim; ++a) {
        n[a] = n_in[a];
        p[a] = p_in[a];
        N *= n[a];
    }
    const int ntiles = p[0] * p[1] * p[2];
    size_t b = (size_t)(2 * dim + 1) * 8 * N + sizeof(TileDesc) * ntiles;        // diagonals, tiles
    b += 8 * 8 * (size_t)N + sizeof(double) * kRedBlocks * 64 + sizeof(double) * 64; // ensure_work
    if (kind != PSW_SSOR && kind != PSW_ILU0) return b;
    const Store st = store_of(prec);
    const size_t eb = store_bytes(st);
    b += (size_t)(2 * dim) * eb * N + eb * N + 8 * (size_t)N; // couplings, pivots, FP64 pivots
    int R, lxmax, lymax;
    if (fast_shape(dim, n, p, prec, lds_limit, R, lxmax, lymax)) {
        const Fast2dPlan pl = fast2d_plan(n, p, R, eb);
        b += 3 * sizeof(int64_t) * ntiles + sizeof(int) * (size_t)pl.otab;
        b += 4 * (3 * eb * (size_t)pl.t + eb * (size_t)(pl.f + 8));
    }
    if (dim == 3 && prec != PSW_F64) {
        std::vector<int> lo[3], len[3];
        PassGeom g{};
        g.dim = 3;
        g.ntiles = ntiles;
        for (int a = 0; a < 3; ++a) {
            g.n[a] = n[a];
            g.sig[a] = 1;
            partition(n[a], p[a], lo[a], len[a]);
        }
        const int l1max = *std::max_element(len[1].begin(), len[1].end());
        const int l2max = *std::max_element(len[2].begin(), len[2].end());
        g.cmax = l1max * l2max;
        g.l1max = l1max;
        g.l2max = l2max;
        const int len0max = *std::max_element(len[0].begin(), len[0].end());
        if (g.cmax <= 1024 && tile3_lds_bytes(g, len0max, sizeof(float)) <= lds_limit) {
            b += sizeof(int64_t) * ntiles + 4 * pack3_slot_bytes(st) * (size_t)tile3_slots(n, p);
            const int64_t fi = faces3_image_elems(g, len0max, lds_limit);
            const int64_t ei = end_faces3_image_elems(g, len0max, lds_limit);
            b += 2 * sizeof(float) * (size_t)std::max<int64_t>(fi, 0) + 2 * sizeof(float) * (size_t)std::max<int64_t>(ei, 0);
            b += 8 * (size_t)N; // the transposed chain's output (CG on the LDS-tile passes)
        }
    }
    return b;
}

size_t devbuf_bytes(const DevBuf &d) { return d.p ? d.bytes : 0; }

// device bytes a problem holds now (its DevBufs)
size_t problem_device_bytes(const psw_problem *P) {
    size_t b = devbuf_bytes(P->tiles) + devbuf_bytes(P->partials) + devbuf_bytes(P->scal);
    for (const DevBuf &d : P->diag) b += devbuf_bytes(d);
    for (const DevBuf *d : {&P->w_r, &P->w_z, &P->w_p, &P->w_q, &P->w_t, &P->w_y, &P->w_y2, &P->w_z1, &P->w_y3,
                            &P->gm_V, &P->gm_Z, &P->gm_h})
        b += devbuf_bytes(*d);
    for (const PrecState &S : P->pc) {
        for (const DevBuf &d : S.diag) b += devbuf_bytes(d);
        b += devbuf_bytes(S.piv) + devbuf_bytes(S.piv64) + devbuf_bytes(S.toff) + devbuf_bytes(S.foff) +
             devbuf_bytes(S.otab) + devbuf_bytes(S.ooff) + devbuf_bytes(S.t3off);
        for (const FastPassBuf &f : S.fp)
            b += devbuf_bytes(f.inv) + devbuf_bytes(f.ax) + devbuf_bytes(f.ay) + devbuf_bytes(f.face);
        for (const DevBuf &d : S.t3pk) b += devbuf_bytes(d);
        for (const DevBuf &d : S.f3img) b += devbuf_bytes(d);
        for (const DevBuf &d : S.e3img) b += devbuf_bytes(d);
    }
    const StatState &T = P->stat;
    b += devbuf_bytes(T.toff) + devbuf_bytes(T.foff) + devbuf_bytes(T.otab) + devbuf_bytes(T.ooff);
    for (const FastPassBuf &f : T.fp)
        b += devbuf_bytes(f.inv) + devbuf_bytes(f.ax) + devbuf_bytes(f.ay) + devbuf_bytes(f.face);
    return b;
}

// one half-sweep; which: 0 fwd (N1), 1 bwd (N2, scaled by c), 2 (Piv-N2)^-T, 3 (Piv-N1)^-T
Fast2dPass fast_pass_desc(psw_problem *P, PrecState &S, int which) {
    int sig[3];
    pass_sig(P, which, sig);
    Fast2dPass fp{};
    fp.g = geom(P, sig);
    fp.R = S.R;
    fp.coupled = which <= 1;
    fp.lxmax = S.lxmax;
    fp.lymax = S.lymax;
    fp.s_inv = S.fp[which].inv.p;
    fp.s_ax = S.fp[which].ax.p;
    fp.s_ay = S.fp[which].ay.p;
    fp.face = S.fp[which].face.p;
    fp.toff = S.toff.as<int64_t>();
    fp.foff = S.foff.as<int64_t>();
    fp.otab = S.otab.as<int>();
    fp.ooff = S.ooff.as<int64_t>();
    return fp;
}

// pipelined pass `which` over all tiles (for the end-coupled passes 2, 3: the uncoupled interior only)
psw_status fast_pass(psw_problem *P, psw_precond kind, int which, const void *in, bool in_f64, bool scale_by_piv,
                     void *out, bool out_f64, double cscale, const double *add, double cadd, hipStream_t st) {
    PrecState &S = P->pc[kind];
    const Fast2dPass fp = fast_pass_desc(P, S, which);
    PassTiming &T = P->timing[which];
    const bool timed = T.on && (T.calls++ % PassTiming::kStride) == 0 && T.used < PassTiming::kPool;
    if (timed) HIPCHK(hipEventRecord(T.ev[2 * T.used], st));
    HIPCHK(launch_fast2d(fp, store_of(P->prec), in, in_f64, scale_by_piv, out, out_f64, which <= 1 ? cscale : 1.0,
                         add, cadd, st));
    if (timed) {
        HIPCHK(hipEventRecord(T.ev[2 * T.used + 1], st));
        ++T.used;
    }
    return PSW_OK;
}

// the coupled end faces and cross points of end-coupled pass `which` (2 or 3), after its interior
psw_status fast_end(psw_problem *P, psw_precond kind, int which, const void *in, bool in_f64, bool scale_by_piv,
                    void *out, bool out_f64, hipStream_t st) {
    PrecState &S = P->pc[kind];
    int sig[3];
    pass_sig(P, which, sig);
    const PassGeom g = geom(P, sig);
    const void *d[7];
    for (int k = 0; k < 7; ++k) d[k] = S.diag[k].p;
    HIPCHK(launch_end_faces2d_fast(g, store_of(P->prec), d, S.piv.p, in, in_f64, scale_by_piv, out, out_f64,
                                   std::max(S.lxmax, S.lymax), st));
    return PSW_OK;
}

psw_status half(psw_problem *P, psw_precond kind, int which, const void *in, bool in_f64, bool scale_by_piv,
                void *out, bool out_f64, double cscale, hipStream_t st) {
    PrecState &S = P->pc[kind];
    Store s = store_of(P->prec);
    int sig[3];
    pass_sig(P, which, sig);
    PassGeom g = geom(P, sig);
    const void *d[7];
    for (int k = 0; k < 7; ++k) d[k] = S.diag[k].p;
    if (S.fast) {
        psw_status ps = fast_pass(P, kind, which, in, in_f64, scale_by_piv, out, out_f64, cscale, nullptr, 0.0, st);
        if (ps || which <= 1) return ps;
        return fast_end(P, kind, which, in, in_f64, scale_by_piv, out, out_f64, st);
    }
    if (S.tile3) {
        // the coupled faces read the coefficient part of their records from the images of tile3_setup
        void *fimg = which <= 1 && S.f3ok[which] ? S.f3img[which].p : nullptr;
        HIPCHK(launch_tile3(g, s, which <= 1, d, S.piv.p, S.t3pk[which].p, S.t3off.as<int64_t>(), S.len0max, in,
                            in_f64, scale_by_piv, out, out_f64, which <= 1 ? cscale : 1.0, fimg, st));
        if (which >= 2)
            HIPCHK(launch_end_fixups3(g, s, d, S.piv.p, in, in_f64, scale_by_piv, out, out_f64, S.len0max,
                                      S.e3ok[which - 2] ? S.e3img[which - 2].p : nullptr, st));
        return PSW_OK;
    }
    if (which <= 1)
        HIPCHK(launch_half_start(g, s, d, S.piv.p, in, in_f64, scale_by_piv, out, out_f64, cscale, st));
    else
        HIPCHK(launch_half_end(g, s, d, S.piv.p, in, in_f64, scale_by_piv, out, out_f64, st));
    return PSW_OK;
}

// The symmetric form in two pieces for the CG loop (pipelined 2D passes only):
// z1 = c (backward pass) and z2 = the transposed pair with its end faces, so
// that z = 0.5 z1 + 0.5 c z2, formed later inside the kernels that read z.
// Each pass has one workgroup per tile that holds the tile in LDS, so a pass
// fills the chip by itself and two passes side by side only time-share it;
// all passes therefore run on st, ordered so that consecutive passes share
// their input (the forward and first transposed passes both read r; the
// backward pass reads the forward pass's output right after it is written).
psw_status precond_sym_split(psw_problem *P, psw_precond kind, const double *r, double *z1, double *z2,
                             hipStream_t st) {
    PrecState &S = P->pc[kind];
    if (!S.fast) return PSW_ENOTSUP;
    const bool f64 = P->prec == PSW_F64;
    void *y1 = P->w_y.p, *y2 = P->w_y2.p;
    psw_status ps;
    if ((ps = fast_pass(P, kind, 2, r, true, false, y2, f64, 1.0, nullptr, 0.0, st))) return ps;
    if ((ps = fast_pass(P, kind, 0, r, true, false, y1, f64, 1.0, nullptr, 0.0, st))) return ps;
    if ((ps = fast_pass(P, kind, 1, y1, f64, true, z1, true, S.c, nullptr, 0.0, st))) return ps;
    if ((ps = fast_end(P, kind, 2, r, true, false, y2, f64, st))) return ps;
    if ((ps = fast_pass(P, kind, 3, y2, f64, true, z2, true, 1.0, nullptr, 0.0, st))) return ps;
    return fast_end(P, kind, 3, y2, f64, true, z2, true, st);
}

// The symmetric form in two pieces on the 3D LDS-tile passes: z1 = c (backward)(forward) r in
// FP64 and z2 = the transposed pair in the sweep precision, so that z = 0.5 z1 + 0.5 c z2.  The two
// chains are independent; the transposed pair runs on the side stream beside the other, with the
// same operations and intermediates as one after the other.  st has joined on return.
psw_status precond_sym_split3(psw_problem *P, psw_precond kind, const double *r, double *z1, const void **z2,
                              hipStream_t st) {
    PrecState &S = P->pc[kind];
    if (!S.tile3) return PSW_ENOTSUP;
    if (!P->side.ensure()) return PSW_EDEVICE;
    if (!P->w_y3.ensure(sizeof(double) * (size_t)P->N)) return PSW_ENOMEM;
    const bool f64 = P->prec == PSW_F64;
    void *y = P->w_y.p, *y2 = P->w_y2.p, *y3 = P->w_y3.p;
    hipStream_t ss = P->side.s;
    psw_status ps;
    HIPCHK(hipEventRecord(P->side.fork, st));
    HIPCHK(hipStreamWaitEvent(ss, P->side.fork, 0));
    if ((ps = half(P, kind, 2, r, true, false, y2, f64, 1.0, ss))) return ps;
    if ((ps = half(P, kind, 3, y2, f64, true, y3, f64, 1.0, ss))) return ps;
    HIPCHK(hipEventRecord(P->side.join, ss));
    if ((ps = half(P, kind, 0, r, true, false, y, f64, 1.0, st))) return ps;
    if ((ps = half(P, kind, 1, y, f64, true, z1, true, S.c, st))) return ps;
    HIPCHK(hipStreamWaitEvent(st, P->side.join, 0));
    *z2 = y3;
    return PSW_OK;
}

psw_status precond_apply(psw_problem *P, psw_precond kind, int symmetric, const double *r, double *z,
                         hipStream_t st) {
    if (kind == PSW_NONE) {
        HIPCHK(hipMemcpyAsync(z, r, sizeof(double) * P->N, hipMemcpyDeviceToDevice, st));
        return PSW_OK;
    }
    psw_status ps = precond_setup(P, kind, st);
    if (ps) return ps;
    if ((ps = ensure_work(P))) return ps;
    PrecState &S = P->pc[kind];
    const bool f64 = P->prec == PSW_F64;
    void *y = P->w_y.p; // intermediate in sweep precision
    if (!symmetric) {
        if ((ps = half(P, kind, 0, r, true, false, y, f64, 1.0, st))) return ps;
        return half(P, kind, 1, y, f64, true, z, true, S.c, st);
    }
    double *z1 = P->w_z1.as<double>();
    if (S.fast) {
        // z = (M^-1 r + M^-T r) / 2.  The transposed pass over r goes first so that its end
        // faces (a small, latency-bound kernel) run on the side stream beside the forward pass;
        // the backward pass finishes with the combination.
        if (!P->side.ensure()) return PSW_EDEVICE;
        void *y1 = P->w_y.p, *y2 = P->w_y2.p;
        if ((ps = fast_pass(P, kind, 2, r, true, false, y2, f64, 1.0, nullptr, 0.0, st))) return ps;
        HIPCHK(hipEventRecord(P->side.fork, st));
        HIPCHK(hipStreamWaitEvent(P->side.s, P->side.fork, 0));
        if ((ps = fast_end(P, kind, 2, r, true, false, y2, f64, P->side.s))) return ps;
        HIPCHK(hipEventRecord(P->side.join, P->side.s));
        if ((ps = fast_pass(P, kind, 0, r, true, false, y1, f64, 1.0, nullptr, 0.0, st))) return ps;
        HIPCHK(hipStreamWaitEvent(st, P->side.join, 0));
        if ((ps = fast_pass(P, kind, 3, y2, f64, true, z1, true, 1.0, nullptr, 0.0, st))) return ps;
        if ((ps = fast_end(P, kind, 3, y2, f64, true, z1, true, st))) return ps;
        return fast_pass(P, kind, 1, y1, f64, true, z, true, S.c, z1, 0.5 * S.c, st);
    }
    if (S.tile3) {
        const void *y3 = nullptr;
        if ((ps = precond_sym_split3(P, kind, r, z1, &y3, st))) return ps;
        HIPCHK(launch_scale_add(z, z1, 0.5, y3, f64, 0.5 * S.c, P->N, st));
        return PSW_OK;
    }
    if ((ps = half(P, kind, 0, r, true, false, y, f64, 1.0, st))) return ps;
    if ((ps = half(P, kind, 1, y, f64, true, z1, true, S.c, st))) return ps;
    void *y2 = P->w_y2.p;
    if ((ps = half(P, kind, 2, r, true, false, y2, f64, 1.0, st))) return ps;
    if ((ps = half(P, kind, 3, y2, f64, true, y, f64, 1.0, st))) return ps;
    HIPCHK(launch_scale_add(z, z1, 0.5, y, f64, 0.5 * S.c, P->N, st));
    return PSW_OK;
}

double now_ms() {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

psw_status host_norm(psw_problem *P, const double *x, double *out, hipStream_t st) {
    double *s = P->scal.as<double>();
    HIPCHK(launch_dot(x, x, P->N, P->partials.as<double>(), s + 10, st));
    double h = 0;
    HIPCHK(hipMemcpyAsync(&h, s + 10, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    *out = std::sqrt(h);
    return PSW_OK;
}

// One decomposed SOR sweep u_out <- sweep(u_in) at schedule step `it`.  2D problems whose tiles fit
// the pipelined pass: the right-hand side f + (1/w - 1) a^P u_in + N2 u_in into w_z, then the
// start-coupled pass with pivots a^P / w of the step's direction map; else the level kernel.
psw_status sweep_once(psw_problem *P, int64_t it, const double *u_in, const double *f, double *u_out,
                      hipStream_t st) {
    int sig[3];
    sched_sig(P, it, sig);
    const double *d[7];
    diag64(P, d);
    if (P->kd == 2 && !P->force_generic) {
        if (!P->stat.ready) {
            psw_status ps = stat_setup(P, st);
            if (ps) return ps;
        }
        if (P->stat.fast) {
            psw_status ps = ensure_work(P);
            if (ps) return ps;
            const int c = sched_step(P, it);
            StatState &S = P->stat;
            double *rhs = P->w_z.as<double>();
            HIPCHK(launch_sor_rhs2d(P->n, P->p, sig, d, P->omega, f, u_in, rhs, st));
            Fast2dPass fp{};
            fp.g = geom(P, sig);
            fp.R = S.R;
            fp.coupled = true;
            fp.lxmax = S.lxmax;
            fp.lymax = S.lymax;
            fp.s_inv = S.fp[c].inv.p;
            fp.s_ax = S.fp[c].ax.p;
            fp.s_ay = S.fp[c].ay.p;
            fp.face = S.fp[c].face.p;
            fp.toff = S.toff.as<int64_t>();
            fp.foff = S.foff.as<int64_t>();
            fp.otab = S.otab.as<int>();
            fp.ooff = S.ooff.as<int64_t>();
            HIPCHK(launch_fast2d(fp, Store::F64, rhs, true, false, u_out, true, 1.0, nullptr, 0.0, st));
            return PSW_OK;
        }
    }
    HIPCHK(launch_sweep_stationary(geom(P, sig), d, P->omega, u_in, f, u_out, st));
    return PSW_OK;
}

// One restricted-overlap sweep (widened boxes of P->overlap points) at schedule step `it`.
psw_status sweep_restricted(psw_problem *P, int64_t it, const double *u_in, const double *f, double *u_out,
                            hipStream_t st) {
    int sig[3];
    sched_sig(P, it, sig);
    const PassGeom g = geom(P, sig);
    int lenmax[3] = {1, 1, 1};
    for (int a = 0; a < P->dim; ++a) {
        std::vector<int> lo, len;
        partition(P->n[a], P->p[a], lo, len);
        lenmax[a] = *std::max_element(len.begin(), len.end());
    }
    const size_t lds = ras_lds_bytes(g, lenmax, P->overlap, P->lds_limit);
    if (!lds) return PSW_ENOTSUP;
    const double *d[7];
    diag64(P, d);
    HIPCHK(launch_ras(g, d, P->omega, P->overlap, lds, u_in, f, u_out, st));
    return PSW_OK;
}

psw_status solve_stationary(psw_problem *P, double rtol, int64_t maxit, const double *f, double *u, psw_info *info,
                            hipStream_t st, bool restricted = false) {
    psw_status ps = ensure_work(P);
    if (ps) return ps;
    if ((ps = check_lds(P, 8))) return ps;
    const double *d[7];
    diag64(P, d);
    double nf;
    if ((ps = host_norm(P, f, &nf, st))) return ps;
    if (nf == 0.0) nf = 1.0;
    double *tmp = P->w_t.as<double>(), *res = P->w_r.as<double>();
    double rel = 0;
    int64_t it = 0;
    bool conv = false;
    for (it = 0; it < maxit;) {
        if ((ps = restricted ? sweep_restricted(P, it, u, f, tmp, st) : sweep_once(P, it, u, f, tmp, st))) return ps;
        HIPCHK(hipMemcpyAsync(u, tmp, sizeof(double) * P->N, hipMemcpyDeviceToDevice, st));
        ++it;
        HIPCHK(launch_residual(P->kd, P->n, d, f, u, res, st));
        double nr;
        if ((ps = host_norm(P, res, &nr, st))) return ps;
        rel = nr / nf;
        if (!std::isfinite(rel)) return PSW_EBREAKDOWN;
        if (rel <= rtol) {
            conv = true;
            break;
        }
    }
    if (info) {
        info->iters = it;
        info->relres = rel;
        info->converged = conv;
    }
    return conv ? PSW_OK : PSW_ENOCONV;
}

// CG iterations on a 2D grid with r = f - A x already in w_r.  Per iteration:
// the fused step (p, deferred x update, q = A p, p.q partials), the r update
// with its r.r partials, the preconditioner and the r.z partials.  p alternates
// between w_p and w_t; the last step's x update is applied on exit.
psw_status cg2d_fused(psw_problem *P, psw_precond kind, bool split, double rtol, int64_t maxit, double nf, double *x,
                      int64_t &it, bool &conv, hipStream_t st) {
    const double *d[7];
    diag64(P, d);
    const int64_t N = P->N;
    double *r = P->w_r.as<double>(), *z = P->w_z.as<double>(), *q = P->w_q.as<double>();
    double *pa = P->w_p.as<double>(), *pb = P->w_t.as<double>();
    double *z2 = split ? P->w_z1.as<double>() : nullptr;
    const double hc = split ? 0.5 * P->pc[kind].c : 0.0;
    double *s = P->scal.as<double>();
    double *s_rz = s + 0, *s_rz2 = s + 1;
    double *part = P->partials.as<double>();
    double *part_pq = part + kRedBlocks, *part_rz = part + 2 * kRedBlocks, *out = part + 3 * kRedBlocks;
    int npq = 0;
    psw_status ps;
    // z from r, then its r.z partials
    auto precond = [&]() -> psw_status {
        if (split) {
            psw_status e = precond_sym_split(P, kind, r, z, z2, st);
            if (e) return e;
            HIPCHK(launch_dot_partial_zz(r, z, z2, hc, N, part_rz, st));
        } else {
            const double *zz = r;
            if (kind != PSW_NONE) {
                psw_status e = precond_apply(P, kind, 1, r, z, st);
                if (e) return e;
                zz = z;
            }
            HIPCHK(launch_dot_partial(r, zz, N, part_rz, st));
        }
        return PSW_OK;
    };
    const double *z1 = (split || kind != PSW_NONE) ? z : r;
    if ((ps = precond())) return ps;
    if (!P->hs.ensure()) return PSW_ENOMEM;
    double *h = P->hs.p, *hdev = nullptr;
    HIPCHK(hipHostGetDevicePointer((void **)&hdev, h, 0));
    PassTiming &T = P->timing[4];
    while (it < maxit) {
        // measurement aid (which = 4): events around every kStride-th fused step
        const bool timed = T.on && (T.calls++ % PassTiming::kStride) == 0 && T.used < PassTiming::kPool;
        if (timed) HIPCHK(hipEventRecord(T.ev[2 * T.used], st));
        HIPCHK(launch_cg_pq2d(P->n[0], P->n[1], d, z1, z2, hc, pa, pb, q, x, part_rz, s_rz2, s_rz, out + 1, it == 0,
                              part_pq, &npq, P->sym, st));
        if (timed) {
            HIPCHK(hipEventRecord(T.ev[2 * T.used + 1], st));
            ++T.used;
        }
        std::swap(pa, pb);
        std::swap(s_rz, s_rz2);
        // p.q and the r.r partials also go straight to pinned host memory, read behind an event;
        // the next preconditioner is queued before the host waits for them, so the device stays
        // busy during the test
        HIPCHK(launch_cg_r(r, q, s_rz, part_pq, npq, out, N, hdev, st));
        ++it;
        HIPCHK(hipEventRecord(P->hs.ev, st));
        if ((ps = precond())) return ps;
        HIPCHK(hipEventSynchronize(P->hs.ev));
        double rr = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) rr += h[2 + b];
        if (!(h[0] > 0.0) || !std::isfinite(rr)) {
            (void)hipStreamSynchronize(st);
            return PSW_EBREAKDOWN;
        }
        if (std::sqrt(rr) / nf <= rtol) {
            conv = true;
            break;
        }
    }
    if (it > 0) HIPCHK(launch_axpy_dev(x, out + 1, pa, N, st));
    return PSW_OK;
}

// The same loop on a 3D grid with the fused 3D step (k_cg_pq3d).  With the LDS-tile passes in
// FP32/BF16 the preconditioned residual stays in two pieces, z = 0.5 z1 + 0.5 c z2 with z2 the
// FP32 output of the transposed pair, formed inside the kernels that read it.
psw_status cg3d_fused(psw_problem *P, psw_precond kind, double rtol, int64_t maxit, double nf, double *x,
                      int64_t &it, bool &conv, hipStream_t st) {
    const double *d[7];
    diag64(P, d);
    const int64_t N = P->N;
    double *r = P->w_r.as<double>(), *z = P->w_z.as<double>(), *q = P->w_q.as<double>();
    double *pa = P->w_p.as<double>(), *pb = P->w_t.as<double>();
    const bool split3 = kind != PSW_NONE && P->pc[kind].tile3 && P->prec != PSW_F64;
    const double hc = split3 ? 0.5 * P->pc[kind].c : 0.0;
    const float *z2f = nullptr;
    double *s = P->scal.as<double>();
    double *s_rz = s + 0, *s_rz2 = s + 1;
    double *part = P->partials.as<double>();
    // the fused step writes up to kCgPq3dMaxBlocks p.q partials: their own region, after out
    double *part_rz = part + 2 * kRedBlocks, *out = part + 3 * kRedBlocks, *part_pq = part + 5 * kRedBlocks;
    static_assert(5 * kRedBlocks + kCgPq3dMaxBlocks <= 64 * kRedBlocks, "partials region");
    int npq = 0;
    psw_status ps;
    // z from r, then its r.z partials
    auto precond = [&]() -> psw_status {
        if (split3) {
            const void *zp = nullptr;
            psw_status e = precond_sym_split3(P, kind, r, z, &zp, st);
            if (e) return e;
            z2f = (const float *)zp;
            HIPCHK(launch_dot_partial_zf(r, z, z2f, hc, N, part_rz, st));
        } else {
            const double *zz = r;
            if (kind != PSW_NONE) {
                psw_status e = precond_apply(P, kind, 1, r, z, st);
                if (e) return e;
                zz = z;
            }
            HIPCHK(launch_dot_partial(r, zz, N, part_rz, st));
        }
        return PSW_OK;
    };
    const double *z1 = kind != PSW_NONE ? z : r;
    if ((ps = precond())) return ps;
    if (!P->hs.ensure()) return PSW_ENOMEM;
    double *h = P->hs.p, *hdev = nullptr;
    HIPCHK(hipHostGetDevicePointer((void **)&hdev, h, 0));
    while (it < maxit) {
        HIPCHK(launch_cg_pq3d(P->n, d, z1, split3 ? z2f : nullptr, hc, pa, pb, q, x, part_rz, s_rz2, s_rz, out + 1,
                              it == 0, part_pq, &npq, P->sym, st));
        std::swap(pa, pb);
        std::swap(s_rz, s_rz2);
        // p.q and the r.r partials go straight to pinned host memory, read behind an event; the
        // next preconditioner is queued before the host waits for them
        HIPCHK(launch_cg_r(r, q, s_rz, part_pq, npq, out, N, hdev, st));
        ++it;
        HIPCHK(hipEventRecord(P->hs.ev, st));
        if ((ps = precond())) return ps;
        HIPCHK(hipEventSynchronize(P->hs.ev));
        double rr = 0.0;
        for (int b = 0; b < kRedBlocks; ++b) rr += h[2 + b];
        if (!(h[0] > 0.0) || !std::isfinite(rr)) {
            (void)hipStreamSynchronize(st);
            return PSW_EBREAKDOWN;
        }
        if (std::sqrt(rr) / nf <= rtol) {
            conv = true;
            break;
        }
    }
    if (it > 0) HIPCHK(launch_axpy_dev(x, out + 1, pa, N, st));
    return PSW_OK;
}

psw_status solve_cg(psw_problem *P, psw_precond kind, double rtol, int64_t maxit, const double *f, double *x,
                    psw_info *info, hipStream_t st) {
    psw_status ps = ensure_work(P);
    if (ps) return ps;
    if (kind != PSW_NONE && (ps = precond_setup(P, kind, st))) return ps;
    const double *d[7];
    diag64(P, d);
    double *r = P->w_r.as<double>();
    double nf;
    if ((ps = host_norm(P, f, &nf, st))) return ps;
    if (nf == 0.0) nf = 1.0;
    HIPCHK(launch_residual(P->kd, P->n, d, f, x, r, st));
    double nr;
    if ((ps = host_norm(P, r, &nr, st))) return ps;
    double rel = nr / nf;
    int64_t it = 0;
    bool conv = rel <= rtol;
    if (!conv) {
        // with the pipelined 2D passes the preconditioned residual stays in two pieces,
        // z = 0.5 z1 + 0.5 c z2, formed inside the two kernels that read it
        const bool split = kind != PSW_NONE && P->pc[kind].fast;
        ps = P->kd == 2 ? cg2d_fused(P, kind, split, rtol, maxit, nf, x, it, conv, st)
                        : cg3d_fused(P, kind, rtol, maxit, nf, x, it, conv, st);
        if (ps) return ps;
    }
    // true residual at exit
    HIPCHK(launch_residual(P->kd, P->n, d, f, x, r, st));
    if ((ps = host_norm(P, r, &nr, st))) return ps;
    if (info) {
        info->iters = it;
        info->relres = nr / nf;
        info->converged = conv;
    }
    return conv ? PSW_OK : PSW_ENOCONV;
}

psw_status solve_fgmres(psw_problem *P, psw_precond kind, double rtol, int64_t maxit, int m, const double *f,
                        double *x, psw_info *info, hipStream_t st) {
    psw_status ps = ensure_work(P);
    if (ps) return ps;
    if (kind != PSW_NONE && (ps = precond_setup(P, kind, st))) return ps;
    if (m < 1) m = 30;
    if (m > 60) m = 60;
    const int64_t N = P->N;
    if (!P->gm_V.ensure(sizeof(double) * (size_t)N * (m + 1)) || !P->gm_Z.ensure(sizeof(double) * (size_t)N * m) ||
        !P->gm_h.ensure(sizeof(double) * 128))
        return PSW_ENOMEM;
    const double *d[7];
    diag64(P, d);
    double *V = P->gm_V.as<double>(), *Z = P->gm_Z.as<double>(), *hd = P->gm_h.as<double>();
    double *r = P->w_r.as<double>(), *w = P->w_q.as<double>();
    double *part = P->partials.as<double>();
    double nf;
    if ((ps = host_norm(P, f, &nf, st))) return ps;
    if (nf == 0.0) nf = 1.0;
    int64_t it = 0;
    bool conv = false;
    double rel = 1.0;
    std::vector<double> H((m + 1) * m), cs(m), sn(m), g(m + 1), y(m), hv(m + 1);
    while (it < maxit) {
        HIPCHK(launch_residual(P->kd, P->n, d, f, x, r, st));
        double beta;
        if ((ps = host_norm(P, r, &beta, st))) return ps;
        rel = beta / nf;
        if (!std::isfinite(rel)) return PSW_EBREAKDOWN;
        if (rel <= rtol) {
            conv = true;
            break;
        }
        HIPCHK(launch_copy_scaled(V, r, 1.0 / beta, N, st));
        std::fill(H.begin(), H.end(), 0.0);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int k_used = 0;
        for (int k = 0; k < m && it < maxit; ++k) {
            double *Vk = V + (size_t)k * N, *Zk = Z + (size_t)k * N;
            if ((ps = precond_apply(P, kind, 0, Vk, Zk, st))) return ps;
            HIPCHK(krylov_spmv(P, d, Zk, w, st));
            // classical Gram-Schmidt, two passes
            for (int pass = 0; pass < 2; ++pass) {
                HIPCHK(launch_multi_dot(V, w, k + 1, N, part, hd, st));
                HIPCHK(hipMemcpyAsync(hv.data(), hd, sizeof(double) * (k + 1), hipMemcpyDeviceToHost, st));
                HIPCHK(hipStreamSynchronize(st));
                for (int i = 0; i <= k; ++i) {
                    H[i * m + k] += hv[i];
                    hv[i] = -hv[i];
                }
                HIPCHK(hipMemcpyAsync(hd + 64, hv.data(), sizeof(double) * (k + 1), hipMemcpyHostToDevice, st));
                HIPCHK(launch_multi_axpy(w, V, hd + 64, k + 1, N, true, st));
            }
            double hn;
            if ((ps = host_norm(P, w, &hn, st))) return ps;
            H[(k + 1) * m + k] = hn;
            ++it;
            k_used = k + 1;
            if (hn > 0) HIPCHK(launch_copy_scaled(V + (size_t)(k + 1) * N, w, 1.0 / hn, N, st));
            for (int i = 0; i < k; ++i) {
                double t = cs[i] * H[i * m + k] + sn[i] * H[(i + 1) * m + k];
                H[(i + 1) * m + k] = -sn[i] * H[i * m + k] + cs[i] * H[(i + 1) * m + k];
                H[i * m + k] = t;
            }
            double den = std::hypot(H[k * m + k], H[(k + 1) * m + k]);
            if (!(den > 0)) return PSW_EBREAKDOWN;
            cs[k] = H[k * m + k] / den;
            sn[k] = H[(k + 1) * m + k] / den;
            H[k * m + k] = den;
            H[(k + 1) * m + k] = 0.0;
            g[k + 1] = -sn[k] * g[k];
            g[k] = cs[k] * g[k];
            rel = std::fabs(g[k + 1]) / nf;
            if (rel <= rtol || hn == 0.0) break;
        }
        for (int i = k_used - 1; i >= 0; --i) {
            double acc = g[i];
            for (int j = i + 1; j < k_used; ++j) acc -= H[i * m + j] * y[j];
            y[i] = acc / H[i * m + i];
        }
        HIPCHK(hipMemcpyAsync(hd + 64, y.data(), sizeof(double) * k_used, hipMemcpyHostToDevice, st));
        HIPCHK(launch_multi_axpy(x, Z, hd + 64, k_used, N, true, st));
        if (rel <= rtol) {
            conv = true;
            break;
        }
    }
    HIPCHK(launch_residual(P->kd, P->n, d, f, x, r, st));
    double nr;
    if ((ps = host_norm(P, r, &nr, st))) return ps;
    if (info) {
        info->iters = it;
        info->relres = nr / nf;
        info->converged = conv && nr / nf <= rtol * 10;
    }
    return conv ? PSW_OK : PSW_ENOCONV;
}


// ---------------------------------------------------------------- batched CG
// CG with the symmetric preconditioner over a batch of 2D problems whose
// preconditioner runs on the pipelined path.  Each problem keeps its own
// buffers; the batch is a device table of pointers.  Two iterations (one per
// parity of the r.z slot) are captured in a hipGraph and replayed; the host
// reads the number of active problems once per replay group.
struct BatchRun {
    std::vector<BProb> hp;
    std::vector<BTile> tiles[2]; // by rows per lane (R = 1, 2)
    std::vector<BChunk> chunks;
    DevBuf dprobs, dtiles[2], dchunks, partials, count, gflags, gscal;
    size_t lds[2] = {0, 0};
    int facemax = 1;
    Store store = Store::F64;
    bool f64 = true;
    int sig[2] = {1, 1};
    int np = 0, nc = 0;
    SideStream side;
};

bool batch_eligible(psw_problem *P, psw_precond kind) {
    if (P->kd != 2 || !P->has_diag || !P->has_decomp) return false;
    if (kind != PSW_SSOR && kind != PSW_ILU0) return false;
    int R, lx, ly;
    return fast_eligible(P, R, lx, ly);
}

psw_status batch_build(BatchRun &B, int count, psw_problem *const *probs, const double *const *f, double *const *u,
                       psw_precond kind, hipStream_t st) {
    B.np = count;
    B.store = store_of(probs[0]->prec);
    B.f64 = probs[0]->prec == PSW_F64;
    int sig3[3];
    sched_sig(probs[0], 0, sig3);
    B.sig[0] = sig3[0];
    B.sig[1] = sig3[1];
    int chunk = 0;
    for (int i = 0; i < count; ++i) {
        psw_problem *P = probs[i];
        if (P->prec != probs[0]->prec || P->phase != probs[0]->phase) return PSW_ENOTSUP;
        psw_status ps = precond_setup(P, kind, st);
        if (ps) return ps;
        if ((ps = ensure_work(P))) return ps;
        PrecState &S = P->pc[kind];
        if (!S.fast) return PSW_ENOTSUP;
        BProb b{};
        b.n0 = P->n[0];
        b.n1 = P->n[1];
        b.N = P->N;
        for (int w = 0; w < 4; ++w) {
            b.s_inv[w] = S.fp[w].inv.p;
            b.s_ax[w] = S.fp[w].ax.p;
            b.s_ay[w] = S.fp[w].ay.p;
            b.face[w] = S.fp[w].face.p;
        }
        b.toff = S.toff.as<int64_t>();
        b.foff = S.foff.as<int64_t>();
        b.otab = S.otab.as<int>();
        b.ooff = S.ooff.as<int64_t>();
        for (int k = 0; k < 5; ++k) {
            b.diagS[k] = S.diag[k].p;
            b.diag64[k] = P->diag[k].as<double>();
        }
        b.pivS = S.piv.p;
        b.vec[kSlotR] = P->w_r.p;
        b.vec[kSlotZ] = P->w_z.p;
        b.vec[kSlotZ1] = P->w_z1.p;
        b.vec[kSlotY1] = P->w_y.p;
        b.vec[kSlotY2] = P->w_y2.p;
        b.vec[kSlotP] = P->w_p.p;
        b.vec[kSlotQ] = P->w_q.p;
        b.vec[kSlotX] = u[i];
        b.vec[kSlotF] = const_cast<double *>(f[i]);
        b.scal = P->scal.as<double>();
        b.flags = reinterpret_cast<int *>(P->scal.as<double>() + 40);
        b.c = S.c;
        b.chunk0 = chunk;
        for (int64_t s0 = 0; s0 < P->N; s0 += kBatchChunk) {
            BChunk c{};
            c.prob = i;
            c.start = s0;
            c.len = (int)std::min<int64_t>(kBatchChunk, P->N - s0);
            B.chunks.push_back(c);
            ++chunk;
        }
        b.nchunk = chunk - b.chunk0;
        B.hp.push_back(b);
        // tiles in the order of the problem's packed offsets
        std::vector<int> lo0, len0, lo1, len1;
        partition(P->n[0], P->p[0], lo0, len0);
        partition(P->n[1], P->p[1], lo1, len1);
        const int g = S.R - 1;
        int tix = 0;
        for (int s1 = 0; s1 < P->p[1]; ++s1)
            for (int s0 = 0; s0 < P->p[0]; ++s0) {
                BTile t{};
                t.td.lo[0] = lo0[s0];
                t.td.len[0] = len0[s0];
                t.td.par[0] = s0 & 1;
                t.td.lo[1] = lo1[s1];
                t.td.len[1] = len1[s1];
                t.td.par[1] = s1 & 1;
                t.td.lo[2] = 0;
                t.td.len[2] = 1;
                t.td.par[2] = 0;
                t.prob = i;
                t.tix = tix++;
                B.tiles[g].push_back(t);
            }
        size_t elem = B.f64 ? 8 : 4;
        B.lds[g] = std::max(B.lds[g], fast2d_lds_bytes(S.lxmax, S.lymax, S.R, elem));
        B.facemax = std::max(B.facemax, std::max(S.lxmax, S.lymax));
    }
    B.nc = (int)B.chunks.size();
    if (!B.dprobs.ensure(sizeof(BProb) * B.hp.size()) || !B.dchunks.ensure(sizeof(BChunk) * B.chunks.size()) ||
        !B.partials.ensure(sizeof(double) * B.chunks.size()) || !B.count.ensure(sizeof(int) * 4) ||
        !B.gflags.ensure(sizeof(int) * 3 * B.hp.size()) || !B.gscal.ensure(sizeof(double) * 5 * B.hp.size()))
        return PSW_ENOMEM;
    HIPCHK(hipMemcpyAsync(B.dprobs.p, B.hp.data(), sizeof(BProb) * B.hp.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(B.dchunks.p, B.chunks.data(), sizeof(BChunk) * B.chunks.size(), hipMemcpyHostToDevice, st));
    for (int g = 0; g < 2; ++g)
        if (!B.tiles[g].empty()) {
            if (!B.dtiles[g].ensure(sizeof(BTile) * B.tiles[g].size())) return PSW_ENOMEM;
            HIPCHK(hipMemcpyAsync(B.dtiles[g].p, B.tiles[g].data(), sizeof(BTile) * B.tiles[g].size(),
                                  hipMemcpyHostToDevice, st));
        }
    HIPCHK(hipStreamSynchronize(st)); // host tables must outlive the copies
    return PSW_OK;
}

// z = (M^-1 + M^-T) r / 2 for every active problem of the batch
psw_status batch_precond(BatchRun &B, hipStream_t st) {
    // the order of the single-problem symmetric preconditioner: transposed pass over r (its end
    // faces on the side stream, beside the forward pass), forward, second transposed pass and
    // its end faces, then the backward pass, which writes z = 0.5 c (result + z2)
    const BProb *dp = B.dprobs.as<BProb>();
    const int sf[2] = {B.sig[0], B.sig[1]}, sb[2] = {-B.sig[0], -B.sig[1]};
    const bool f64 = B.f64;
    if (!B.side.ensure()) return PSW_EDEVICE;
    for (int g = 0; g < 2; ++g) {
        const int nt = (int)B.tiles[g].size();
        if (!nt) continue;
        HIPCHK(launch_b_fast2d(B.dtiles[g].as<BTile>(), nt, dp, sf, 2, g + 1, B.store, kSlotR, true, kSlotY2, f64, false,
                               false, false, -1, B.lds[g], st));
    }
    HIPCHK(hipEventRecord(B.side.fork, st));
    HIPCHK(hipStreamWaitEvent(B.side.s, B.side.fork, 0));
    for (int g = 0; g < 2; ++g) {
        const int nt = (int)B.tiles[g].size();
        if (!nt) continue;
        HIPCHK(launch_b_end2d(B.dtiles[g].as<BTile>(), nt, dp, sf, B.store, kSlotR, true, kSlotY2, f64, false,
                              B.facemax, B.side.s));
    }
    HIPCHK(hipEventRecord(B.side.join, B.side.s));
    for (int g = 0; g < 2; ++g) {
        const int nt = (int)B.tiles[g].size();
        if (!nt) continue;
        HIPCHK(launch_b_fast2d(B.dtiles[g].as<BTile>(), nt, dp, sf, 0, g + 1, B.store, kSlotR, true, kSlotY1, f64, false,
                               true, false, -1, B.lds[g], st));
    }
    HIPCHK(hipStreamWaitEvent(st, B.side.join, 0));
    for (int g = 0; g < 2; ++g) {
        const int nt = (int)B.tiles[g].size();
        if (!nt) continue;
        HIPCHK(launch_b_fast2d(B.dtiles[g].as<BTile>(), nt, dp, sb, 3, g + 1, B.store, kSlotY2, f64, kSlotZ1, true, true,
                               false, false, -1, B.lds[g], st));
    }
    for (int g = 0; g < 2; ++g) {
        const int nt = (int)B.tiles[g].size();
        if (!nt) continue;
        HIPCHK(launch_b_end2d(B.dtiles[g].as<BTile>(), nt, dp, sb, B.store, kSlotY2, f64, kSlotZ1, true, true, B.facemax,
                              st));
    }
    for (int g = 0; g < 2; ++g) {
        const int nt = (int)B.tiles[g].size();
        if (!nt) continue;
        HIPCHK(launch_b_fast2d(B.dtiles[g].as<BTile>(), nt, dp, sb, 1, g + 1, B.store, kSlotY1, f64, kSlotZ, true, true,
                               true, true, kSlotZ1, B.lds[g], st));
    }
    return PSW_OK;
}

psw_status batch_iteration(BatchRun &B, int par, double rtol2, int64_t maxit, hipStream_t st) {
    const BProb *dp = B.dprobs.as<BProb>();
    const BChunk *dc = B.dchunks.as<BChunk>();
    double *part = B.partials.as<double>();
    HIPCHK(launch_b_spmv(dc, B.nc, dp, kSlotP, kSlotQ, false, st));
    HIPCHK(launch_b_dot(dc, B.nc, dp, B.np, kSlotP, kSlotQ, part, 2, false, st));
    HIPCHK(launch_b_cg_xr(dc, B.nc, dp, B.np, par, part, st));
    HIPCHK(launch_b_check(dp, B.np, rtol2, maxit, st));
    psw_status ps = batch_precond(B, st);
    if (ps) return ps;
    HIPCHK(launch_b_dot(dc, B.nc, dp, B.np, kSlotR, kSlotZ, part, 1 - par, false, st));
    HIPCHK(launch_b_cg_p(dc, B.nc, dp, 1 - par, par, st));
    return PSW_OK;
}

// start of a solve for every problem of B: r = f - A x, f.f, r.r, activity,
// z = M r, r.z (parity 0), p = z
psw_status batch_start(BatchRun &B, double rtol2, hipStream_t st) {
    const BProb *dp = B.dprobs.as<BProb>();
    const BChunk *dc = B.dchunks.as<BChunk>();
    double *part = B.partials.as<double>();
    HIPCHK(launch_b_activate(dp, B.np, st));
    HIPCHK(launch_b_spmv(dc, B.nc, dp, kSlotX, kSlotR, true, st));
    HIPCHK(launch_b_dot(dc, B.nc, dp, B.np, kSlotF, kSlotF, part, 4, true, st));
    HIPCHK(launch_b_dot(dc, B.nc, dp, B.np, kSlotR, kSlotR, part, 3, true, st));
    HIPCHK(launch_b_init(dp, B.np, rtol2, st));
    psw_status ps = batch_precond(B, st);
    if (ps) return ps;
    HIPCHK(launch_b_dot(dc, B.nc, dp, B.np, kSlotR, kSlotZ, part, 0, false, st));
    HIPCHK(launch_b_copy(dc, B.nc, dp, kSlotZ, kSlotP, st));
    return PSW_OK;
}

// true residuals of every problem of B; fills infos (iterations, status, relres)
psw_status batch_finish(BatchRun &B, psw_info *infos, hipStream_t st) {
    const BProb *dp = B.dprobs.as<BProb>();
    const BChunk *dc = B.dchunks.as<BChunk>();
    double *part = B.partials.as<double>();
    const int count = B.np;
    std::vector<int> fl(3 * count);
    std::vector<double> sc(5 * count);
    // iterations and status before the activity flags are reset for the residual pass
    HIPCHK(launch_b_gather(dp, count, B.gflags.as<int>(), nullptr, st));
    HIPCHK(hipMemcpyAsync(fl.data(), B.gflags.p, sizeof(int) * 3 * count, hipMemcpyDeviceToHost, st));
    HIPCHK(launch_b_activate(dp, count, st));
    HIPCHK(launch_b_spmv(dc, B.nc, dp, kSlotX, kSlotR, true, st));
    HIPCHK(launch_b_dot(dc, B.nc, dp, count, kSlotR, kSlotR, part, 3, true, st));
    HIPCHK(launch_b_gather(dp, count, B.gflags.as<int>(), B.gscal.as<double>(), st));
    HIPCHK(hipMemcpyAsync(sc.data(), B.gscal.p, sizeof(double) * 5 * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (int i = 0; i < count; ++i) {
        const double ff = sc[5 * i + 4] > 0 ? sc[5 * i + 4] : 1.0;
        psw_info inf{};
        inf.iters = fl[3 * i + 1];
        inf.relres = std::sqrt(sc[5 * i + 3] / ff);
        inf.status = fl[3 * i + 2];
        inf.converged = inf.status == PSW_OK;
        infos[i] = inf;
    }
    return PSW_OK;
}

struct StreamHolder {
    hipStream_t s = nullptr;
    ~StreamHolder() {
        if (s) (void)hipStreamDestroy(s);
    }
};

psw_status batch_cg(int count, psw_problem *const *probs, const double *const *f, double *const *u, psw_precond kind,
                    double rtol, int64_t maxit, psw_info *infos, hipStream_t user) {
    const double t0 = now_ms();
    BatchRun B;
    // work on an internal stream (graph capture needs a capturable stream), ordered after the caller's
    StreamHolder sh;
    HIPCHK(hipStreamCreateWithFlags(&sh.s, hipStreamNonBlocking));
    hipStream_t st = sh.s;
    HIPCHK(hipStreamSynchronize(user));
    psw_status ps = batch_build(B, count, probs, f, u, kind, st);
    if (ps) return ps;
    const BProb *dp = B.dprobs.as<BProb>();
    const double rtol2 = rtol * rtol;
    if ((ps = batch_start(B, rtol2, st))) return ps;
    // two iterations in one graph
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIPCHK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    psw_status cap = batch_iteration(B, 0, rtol2, maxit, st);
    if (cap == PSW_OK) cap = batch_iteration(B, 1, rtol2, maxit, st);
    hipError_t ec = hipStreamEndCapture(st, &graph);
    if (cap != PSW_OK || ec != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return cap != PSW_OK ? cap : PSW_EDEVICE;
    }
    if (hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return PSW_EDEVICE;
    }
    int *hcount = nullptr;
    if (hipHostMalloc((void **)&hcount, sizeof(int)) != hipSuccess) {
        (void)hipGraphExecDestroy(exec);
        (void)hipGraphDestroy(graph);
        return PSW_ENOMEM;
    }
    psw_status run = PSW_OK;
    const int per_poll = 8; // graph replays (2 iterations each) between polls
    for (int64_t done = 0; done < maxit + 2; done += 2 * per_poll) {
        for (int k = 0; k < per_poll; ++k)
            if (hipGraphLaunch(exec, st) != hipSuccess) run = PSW_EDEVICE;
        if (run) break;
        if (launch_b_count(dp, B.np, B.count.as<int>(), st) != hipSuccess ||
            hipMemcpyAsync(hcount, B.count.p, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess) {
            run = PSW_EDEVICE;
            break;
        }
        if (*hcount == 0) break;
    }
    (void)hipGraphExecDestroy(exec);
    (void)hipGraphDestroy(graph);
    (void)hipHostFree(hcount);
    if (run) return run;
    std::vector<psw_info> loc(count);
    if ((ps = batch_finish(B, loc.data(), st))) return ps;
    const double t1 = now_ms();
    psw_status worst = PSW_OK;
    for (int i = 0; i < count; ++i) {
        loc[i].t_total_ms = t1 - t0;
        if (infos) infos[i] = loc[i];
        if (loc[i].status != PSW_OK && worst == PSW_OK) worst = (psw_status)loc[i].status;
    }
    return worst;
}


// ---------------------------------------------------------------- autotuner
// Tile shape for a 2D problem size in a batch: candidate tile sides are timed
// on the batched symmetric preconditioner with the problem replicated until
// its tiles fill the device, and the cheapest per problem wins.  Results are
// cached per (n0, n1, precision, preconditioner) for the life of the process.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, std::pair<int, int>> g_tune_cache;

// candidate tile sides, and the subdomain count of an axis of n points for a side
const int kTuneSides[] = {16, 24, 32, 48, 64, 96, 128};
int tune_count(int n, int side) { return std::min(std::max(1, (n + side - 1) / side), std::max(1, n / 2)); }

psw_status tune_candidate(int n0, int n1, psw_prec prec, psw_precond kind, int p0, int p1, double *us,
                          hipStream_t st) {
    const int64_t n[3] = {n0, n1, 1};
    psw_problem *P = nullptr;
    psw_status ps = psw_problem_create(2, n, 5, &P);
    if (ps) return ps;
    struct Closer {
        psw_problem *p;
        ~Closer() { psw_problem_destroy(p); }
    } closer{P};
    // unit coefficients: the tile shape, not the values, sets the cost
    std::vector<double> one((size_t)P->N, 1.0), four((size_t)P->N, 4.0);
    const double *dg[5] = {four.data(), one.data(), one.data(), one.data(), one.data()};
    if ((ps = psw_set_diagonals(P, dg, 0, prec, st))) return ps;
    const double w = 1.0;
    if ((ps = psw_set_relaxation(P, &w, 1))) return ps;
    const int pp[3] = {p0, p1, 1};
    if ((ps = psw_set_decomposition(P, pp, 2, 0))) return ps;
    if (!batch_eligible(P, kind)) return PSW_ENOTSUP;
    const int tiles = p0 * p1;
    const int reps_prob = std::max(1, (2 * 256 + tiles - 1) / tiles);
    std::vector<psw_problem *> probs(reps_prob, P);
    std::vector<const double *> f(reps_prob, nullptr);
    std::vector<double *> u(reps_prob, nullptr);
    if ((ps = ensure_work(P))) return ps;
    for (int i = 0; i < reps_prob; ++i) {
        f[i] = P->w_t.as<double>();
        u[i] = P->w_t.as<double>();
    }
    BatchRun B;
    if ((ps = batch_build(B, reps_prob, probs.data(), f.data(), u.data(), kind, st))) return ps;
    HIPCHK(launch_b_activate(B.dprobs.as<BProb>(), B.np, st));
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    psw_status run = batch_precond(B, st); // warm-up
    const int reps = 3;
    if (!run) {
        (void)hipEventRecord(e0, st);
        for (int k = 0; k < reps && !run; ++k) run = batch_precond(B, st);
        (void)hipEventRecord(e1, st);
    }
    float ms = 0.f;
    if (!run && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        run = PSW_EDEVICE;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (run) return run;
    *us = 1e3 * ms / reps / reps_prob;
    return PSW_OK;
}

psw_status autotune2d(int n0, int n1, psw_prec prec, psw_precond kind, int p[2], double *best_us, hipStream_t st) {
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune_cache.find(std::make_tuple(n0, n1, (int)prec, (int)kind));
        if (it != g_tune_cache.end()) {
            p[0] = it->second.first;
            p[1] = it->second.second;
            if (best_us) *best_us = -1.0;
            return PSW_OK;
        }
    }
    double best = 1e300;
    int bp0 = 0, bp1 = 0;
    for (int side : kTuneSides) {
        int p0 = tune_count(n0, side), p1 = tune_count(n1, side);
        double us = 0;
        psw_status ps = tune_candidate(n0, n1, prec, kind, p0, p1, &us, st);
        if (ps == PSW_ENOTSUP || ps == PSW_EINVAL) continue;
        if (ps) return ps;
        if (us < best) {
            best = us;
            bp0 = p0;
            bp1 = p1;
        }
    }
    if (!bp0) return PSW_ENOTSUP;
    p[0] = bp0;
    p[1] = bp1;
    if (best_us) *best_us = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[std::make_tuple(n0, n1, (int)prec, (int)kind)] = {bp0, bp1};
    return PSW_OK;
}


// ---------------------------------------------------------------- serving
// Requests carry a coefficient field and a right-hand side (host arrays).
// Admission reserves an estimate of the request's device memory against the
// budget.  2D requests join a continuously batched CG: between epochs of an
// even number of iterations, admitted problems are started and joined to the
// active set and converged ones are retired and freed.  3D requests are solved
// one at a time on a second stream, overlapping with the 2D batch.
struct SrvReq {
    uint64_t id = 0;
    int dim = 2;
    int64_t n[3] = {1, 1, 1};
    int64_t N = 0;
    std::vector<double> alpha[3];
    double beta = 0.0;
    std::vector<double> f, u;
    psw_info info{};
    int state = 0; // 0 queued, 1 running, 2 done
    double t_submit = 0, t_admit = 0, t_done = 0;
    size_t bytes = 0;
    psw_problem *P = nullptr;
    DevBuf dx, df, dal[3];
};

// subdomain counts of a served problem: 2D from the tile side that the autotuner chose for the
// size bucket (side <= 0: no answer, 128-point tiles), 3D with 32-point tiles
void srv_decomp(int dim, const int64_t n[3], int side, int p[3]) {
    p[0] = p[1] = p[2] = 1;
    if (dim == 3) {
        for (int a = 0; a < 3; ++a) p[a] = (int)std::max<int64_t>(1, std::min<int64_t>(n[a] / 2, (n[a] + 31) / 32));
        return;
    }
    if (side <= 0) side = 128;
    for (int a = 0; a < 2; ++a)
        p[a] = (int)std::max<int64_t>(1, std::min<int64_t>(n[a] / 2, (n[a] + side - 1) / side));
}

// size bucket of a served 2D problem (the autotuner's cache key)
int srv_bucket(const int64_t n[3]) { return (int)std::max<int64_t>(32, ((n[0] + 32) / 64) * 64); }

// Admission estimate of a request: its problem's device bytes (problem_bytes, for the largest
// footprint among the decompositions the autotuner can pick), the right-hand side and solution,
// the node coefficients held during set-up, and its share of the batch tables.
size_t request_bytes(int dim, const int64_t n[3], psw_prec prec, psw_precond kind, size_t lds_limit) {
    int64_t N = 1, nodes = 1;
    int nn[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) {
        N *= n[a];
        nodes *= n[a] + 2;
        nn[a] = (int)n[a];
    }
    size_t worst = 0;
    int p[3];
    if (dim == 3) {
        srv_decomp(3, n, 0, p);
        worst = problem_bytes(3, nn, p, prec, kind, lds_limit);
    } else {
        const int b = srv_bucket(n);
        srv_decomp(2, n, 0, p);
        worst = problem_bytes(2, nn, p, prec, kind, lds_limit);
        for (int side : kTuneSides) {
            srv_decomp(2, n, std::max(2, b / tune_count(b, side)), p);
            worst = std::max(worst, problem_bytes(2, nn, p, prec, kind, lds_limit));
        }
    }
    const int64_t chunks = (N + kBatchChunk - 1) / kBatchChunk;
    const size_t tables = sizeof(BProb) + (size_t)chunks * (sizeof(BChunk) + sizeof(double)) +
                          (size_t)p[0] * p[1] * p[2] * sizeof(BTile) + 3 * sizeof(int) + 5 * sizeof(double);
    return worst + 2 * sizeof(double) * (size_t)N + (size_t)nodes * 8 * dim + tables;
}

} // namespace

struct psw_server {
    std::mutex mu;
    std::condition_variable cv;
    std::deque<SrvReq *> q2, q3;
    std::map<uint64_t, std::unique_ptr<SrvReq>> reqs;
    size_t budget = 0, used = 0;
    psw_prec prec = PSW_F32;
    psw_precond precond = PSW_SSOR;
    double rtol = 1e-8;
    int64_t maxit = 100000;
    int epoch_iters = 16;
    int max_active = 1024;
    int lanes3d = 4;
    bool stop = false;
    uint64_t next_id = 1;
    int device = 0;
    size_t lds_limit = 65536;
    int64_t n_done = 0;
    std::thread w2;
    std::vector<std::thread> w3;
};

namespace {

// set up a request's problem on the device (assembly, decomposition, preconditioner)
psw_status srv_setup(psw_server *S, SrvReq *r, hipStream_t st) {
    psw_status ps = psw_problem_create(r->dim, r->n, 2 * r->dim + 1, &r->P);
    if (ps) return ps;
    int64_t nodes = 1;
    for (int a = 0; a < r->dim; ++a) nodes *= r->n[a] + 2;
    const double *al[3] = {nullptr, nullptr, nullptr};
    for (int a = 0; a < r->dim; ++a) {
        if (!r->dal[a].ensure(sizeof(double) * nodes)) return PSW_ENOMEM;
        HIPCHK(hipMemcpyAsync(r->dal[a].p, r->alpha[a].data(), sizeof(double) * nodes, hipMemcpyHostToDevice, st));
        al[a] = r->dal[a].as<double>();
    }
    if (!r->df.ensure(sizeof(double) * r->N) || !r->dx.ensure(sizeof(double) * r->N)) return PSW_ENOMEM;
    HIPCHK(hipMemcpyAsync(r->df.p, r->f.data(), sizeof(double) * r->N, hipMemcpyHostToDevice, st));
    HIPCHK(hipMemsetAsync(r->dx.p, 0, sizeof(double) * r->N, st));
    if ((ps = psw_assemble_diffusion(r->P, al, r->beta, S->prec, st))) return ps;
    const double w = 1.0;
    if ((ps = psw_set_relaxation(r->P, &w, 1))) return ps;
    int p[3] = {1, 1, 1};
    int side = 0;
    if (r->dim == 2) {
        // autotuned tile side of the size bucket
        const int b = srv_bucket(r->n);
        int pb[2];
        if (autotune2d(b, b, S->prec, S->precond, pb, nullptr, st) == PSW_OK) side = std::max(2, b / pb[0]);
    }
    srv_decomp(r->dim, r->n, side, p);
    if ((ps = psw_set_decomposition(r->P, p, 2, 0))) return ps;
    if ((ps = precond_setup(r->P, S->precond, st))) return ps;
    HIPCHK(hipStreamSynchronize(st));
    r->alpha[0].clear();
    r->alpha[1].clear();
    r->alpha[2].clear();
    for (int a = 0; a < 3; ++a) r->dal[a].release();
    return PSW_OK;
}

void srv_finish(psw_server *S, SrvReq *r, psw_status st_code, hipStream_t st) {
    r->u.assign((size_t)r->N, 0.0);
    if (r->dx.p) (void)hipMemcpyAsync(r->u.data(), r->dx.p, sizeof(double) * r->N, hipMemcpyDeviceToHost, st);
    (void)hipStreamSynchronize(st);
    // every kernel of this request ran on st, which has drained: free without a device-wide
    // synchronisation, so other lanes' solves keep running
    delete r->P;
    r->P = nullptr;
    r->dx.release();
    r->df.release();
    r->f.clear();
    std::lock_guard<std::mutex> lk(S->mu);
    r->t_done = now_ms();
    if (st_code != PSW_OK) r->info.status = st_code;
    r->info.converged = r->info.status == PSW_OK;
    r->info.t_total_ms = r->t_done - r->t_submit;
    r->state = 2;
    S->used -= r->bytes;
    ++S->n_done;
    S->cv.notify_all();
}

// one request solved alone (host-driven CG)
void srv_solve_one(psw_server *S, SrvReq *r, hipStream_t st) {
    psw_info inf{};
    psw_status ps = psw_solve(r->P, PSW_CG, S->precond, S->rtol, S->maxit, 30, r->df.as<double>(), r->dx.as<double>(),
                              &inf, st);
    r->info = inf;
    srv_finish(S, r, ps, st);
}

void srv_admit(psw_server *S, std::deque<SrvReq *> &q, std::vector<SrvReq *> &out, size_t max_new) {
    std::lock_guard<std::mutex> lk(S->mu);
    while (!q.empty() && out.size() < max_new && S->used + q.front()->bytes <= S->budget) {
        SrvReq *r = q.front();
        q.pop_front();
        S->used += r->bytes;
        r->state = 1;
        r->t_admit = now_ms();
        out.push_back(r);
    }
}

void srv_lane2d(psw_server *S) {
    (void)hipSetDevice(S->device);
    StreamHolder sh;
    if (hipStreamCreateWithFlags(&sh.s, hipStreamNonBlocking) != hipSuccess) return;
    hipStream_t st = sh.s;
    const double rtol2 = S->rtol * S->rtol;
    std::vector<SrvReq *> active;
    std::unique_ptr<BatchRun> B;
    bool dirty = true;
    for (;;) {
        std::vector<SrvReq *> fresh;
        const size_t room = active.size() < (size_t)S->max_active ? S->max_active - active.size() : 0;
        srv_admit(S, S->q2, fresh, room);
        if (active.empty() && fresh.empty()) {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && S->q2.empty()) break;
            S->cv.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        // start the admitted problems
        std::vector<SrvReq *> ok;
        for (SrvReq *r : fresh) {
            psw_status ps = srv_setup(S, r, st);
            if (ps) {
                srv_finish(S, r, ps, st);
            } else if (!batch_eligible(r->P, S->precond)) {
                srv_solve_one(S, r, st); // a shape the batched kernels do not take
            } else {
                ok.push_back(r);
            }
        }
        if (!ok.empty()) {
            std::vector<psw_problem *> pp;
            std::vector<const double *> ff;
            std::vector<double *> uu;
            for (SrvReq *r : ok) {
                pp.push_back(r->P);
                ff.push_back(r->df.as<double>());
                uu.push_back(r->dx.as<double>());
            }
            BatchRun Bn;
            psw_status ps = batch_build(Bn, (int)ok.size(), pp.data(), ff.data(), uu.data(), S->precond, st);
            if (!ps) ps = batch_start(Bn, rtol2, st);
            if (!ps && hipStreamSynchronize(st) != hipSuccess) ps = PSW_EDEVICE;
            if (ps) {
                for (SrvReq *r : ok) srv_finish(S, r, ps, st);
            } else {
                active.insert(active.end(), ok.begin(), ok.end());
                dirty = true;
            }
        }
        if (active.empty()) continue;
        if (dirty) {
            B.reset(new BatchRun());
            std::vector<psw_problem *> pp;
            std::vector<const double *> ff;
            std::vector<double *> uu;
            for (SrvReq *r : active) {
                pp.push_back(r->P);
                ff.push_back(r->df.as<double>());
                uu.push_back(r->dx.as<double>());
            }
            psw_status ps = batch_build(*B, (int)active.size(), pp.data(), ff.data(), uu.data(), S->precond, st);
            if (ps) {
                for (SrvReq *r : active) srv_finish(S, r, ps, st);
                active.clear();
                continue;
            }
            dirty = false;
        }
        // an epoch: an even number of iterations keeps every problem at r.z parity 0
        psw_status ps = PSW_OK;
        for (int k = 0; k < S->epoch_iters && !ps; ++k) ps = batch_iteration(*B, k & 1, rtol2, S->maxit, st);
        std::vector<int> fl(3 * active.size());
        if (!ps && (launch_b_gather(B->dprobs.as<BProb>(), B->np, B->gflags.as<int>(), nullptr, st) != hipSuccess ||
                    hipMemcpyAsync(fl.data(), B->gflags.p, sizeof(int) * fl.size(), hipMemcpyDeviceToHost, st) !=
                        hipSuccess ||
                    hipStreamSynchronize(st) != hipSuccess))
            ps = PSW_EDEVICE;
        if (ps) {
            for (SrvReq *r : active) srv_finish(S, r, ps, st);
            active.clear();
            dirty = true;
            continue;
        }
        // retire the finished problems
        std::vector<SrvReq *> done, keep;
        for (size_t i = 0; i < active.size(); ++i) (fl[3 * i] ? keep : done).push_back(active[i]);
        if (!done.empty()) {
            std::vector<psw_problem *> pp;
            std::vector<const double *> ff;
            std::vector<double *> uu;
            for (SrvReq *r : done) {
                pp.push_back(r->P);
                ff.push_back(r->df.as<double>());
                uu.push_back(r->dx.as<double>());
            }
            BatchRun Bd;
            std::vector<psw_info> inf(done.size());
            psw_status fs = batch_build(Bd, (int)done.size(), pp.data(), ff.data(), uu.data(), S->precond, st);
            if (!fs) fs = batch_finish(Bd, inf.data(), st);
            for (size_t i = 0; i < done.size(); ++i) {
                if (!fs) done[i]->info = inf[i];
                srv_finish(S, done[i], fs ? fs : (psw_status)inf[i].status, st);
            }
            active.swap(keep);
            dirty = true;
        }
    }
}

void srv_lane3d(psw_server *S) {
    (void)hipSetDevice(S->device);
    StreamHolder sh;
    if (hipStreamCreateWithFlags(&sh.s, hipStreamNonBlocking) != hipSuccess) return;
    hipStream_t st = sh.s;
    for (;;) {
        std::vector<SrvReq *> one;
        srv_admit(S, S->q3, one, 1);
        if (one.empty()) {
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->stop && S->q3.empty()) break;
            S->cv.wait_for(lk, std::chrono::milliseconds(2));
            continue;
        }
        SrvReq *r = one[0];
        psw_status ps = srv_setup(S, r, st);
        if (ps) srv_finish(S, r, ps, st);
        else srv_solve_one(S, r, st);
    }
}

} // namespace

// ------------------------------------------------ preconditioner without allocation
// The intermediate vector of the pair form lives in a fixed device array.  Host code never passes
// the array's name to a kernel: it takes the array's device address once per device with
// hipGetSymbolAddress and uses that pointer.
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[64] = {};

// device address of `scratch` on device dev (dev current); nullptr on failure
void *scratch_ptr(int dev) {
    if (dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
} // namespace

// ====================================================================== C ABI
extern "C" {

psw_status psw_server_create(size_t budget_bytes, const psw_server_opts *opts, psw_server **out) {
    if (!out || budget_bytes == 0) return PSW_EINVAL;
    *out = nullptr;
    psw_server *S = new (std::nothrow) psw_server();
    if (!S) return PSW_ENOMEM;
    if (hipGetDevice(&S->device) != hipSuccess) {
        delete S;
        return PSW_EDEVICE;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, S->device) == hipSuccess && lds > 0)
        S->lds_limit = (size_t)lds;
    S->budget = budget_bytes;
    if (opts) {
        if (opts->prec < PSW_F64 || opts->prec > PSW_BF16 || (opts->precond != PSW_SSOR && opts->precond != PSW_ILU0) ||
            !(opts->rtol > 0.0) || opts->maxit < 1) {
            delete S;
            return PSW_EINVAL;
        }
        S->prec = opts->prec;
        S->precond = opts->precond;
        S->rtol = opts->rtol;
        S->maxit = opts->maxit;
        if (opts->epoch_iters > 0) S->epoch_iters = (opts->epoch_iters + 1) & ~1;
        if (opts->max_active > 0) S->max_active = opts->max_active;
        if (opts->lanes3d > 0) S->lanes3d = std::min(opts->lanes3d, 16);
    }
    S->w2 = std::thread(srv_lane2d, S);
    for (int k = 0; k < S->lanes3d; ++k) S->w3.emplace_back(srv_lane3d, S);
    *out = S;
    return PSW_OK;
}

psw_status psw_server_submit(psw_server *S, int dim, const int64_t n[3], const double *const alpha[], double beta,
                             const double *f, uint64_t *ticket) {
    if (!S || !n || !alpha || !f || !ticket || (dim != 2 && dim != 3) || !(beta >= 0.0)) return PSW_EINVAL;
    std::unique_ptr<SrvReq> r(new (std::nothrow) SrvReq());
    if (!r) return PSW_ENOMEM;
    r->dim = dim;
    r->N = 1;
    int64_t nodes = 1;
    for (int a = 0; a < dim; ++a) {
        if (n[a] < 4 || n[a] > (1 << 16) || !alpha[a]) return PSW_EINVAL;
        r->n[a] = n[a];
        r->N *= n[a];
        nodes *= n[a] + 2;
    }
    r->bytes = request_bytes(dim, r->n, S->prec, S->precond, S->lds_limit);
    if (r->bytes > S->budget) return PSW_EBUSY;
    for (int a = 0; a < dim; ++a) r->alpha[a].assign(alpha[a], alpha[a] + nodes);
    r->f.assign(f, f + r->N);
    r->beta = beta;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return PSW_ESTATE;
    r->id = S->next_id++;
    r->t_submit = now_ms();
    SrvReq *raw = r.get();
    S->reqs[raw->id] = std::move(r);
    (dim == 2 ? S->q2 : S->q3).push_back(raw);
    *ticket = raw->id;
    S->cv.notify_all();
    return PSW_OK;
}

psw_status psw_server_request_bytes(psw_server *S, int dim, const int64_t n[3], size_t *bytes) {
    if (!S || !n || !bytes || (dim != 2 && dim != 3)) return PSW_EINVAL;
    for (int a = 0; a < dim; ++a)
        if (n[a] < 4 || n[a] > (1 << 16)) return PSW_EINVAL;
    int64_t nn[3] = {1, 1, 1};
    for (int a = 0; a < dim; ++a) nn[a] = n[a];
    *bytes = request_bytes(dim, nn, S->prec, S->precond, S->lds_limit);
    return PSW_OK;
}

psw_status psw_server_poll(psw_server *S, uint64_t ticket, int wait, int *done, psw_info *info, double *u,
                           double *t_queue_ms) {
    if (!S || !done) return PSW_EINVAL;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return PSW_EINVAL;
    SrvReq *r = it->second.get();
    if (wait) S->cv.wait(lk, [&] { return r->state == 2; });
    *done = r->state == 2;
    if (!*done) return PSW_OK;
    if (info) *info = r->info;
    if (t_queue_ms) *t_queue_ms = r->t_admit - r->t_submit;
    if (u) std::copy(r->u.begin(), r->u.end(), u);
    S->reqs.erase(it); // a finished request is handed out once
    return PSW_OK;
}

psw_status psw_server_destroy(psw_server *S) {
    if (!S) return PSW_EINVAL;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        S->cv.notify_all();
    }
    if (S->w2.joinable()) S->w2.join();
    for (auto &t : S->w3)
        if (t.joinable()) t.join();
    delete S;
    return PSW_OK;
}

psw_status psw_pass_timing_enable(psw_problem *P, int which, int enable) {
    if (!P || which < 0 || which > 4) return PSW_EINVAL;
    DeviceGuard dg(P->device);
    PassTiming &T = P->timing[which];
    P->timing_last = which;
    if (enable && T.ev.empty()) {
        T.ev.assign(2 * PassTiming::kPool, nullptr);
        for (auto &e : T.ev)
            if (hipEventCreate(&e) != hipSuccess) return PSW_EDEVICE;
    }
    T.on = enable != 0;
    T.which = which;
    T.calls = 0;
    T.used = 0;
    return PSW_OK;
}

psw_status psw_pass_timing_of(psw_problem *P, int which, double *mean_ms, int64_t *count) {
    if (!P || !mean_ms || !count || which < 0 || which > 4) return PSW_EINVAL;
    DeviceGuard dg(P->device);
    PassTiming &T = P->timing[which];
    double sum = 0.0;
    for (int64_t i = 0; i < T.used; ++i) {
        float ms = 0.f;
        HIPCHK(hipEventSynchronize(T.ev[2 * i + 1]));
        HIPCHK(hipEventElapsedTime(&ms, T.ev[2 * i], T.ev[2 * i + 1]));
        sum += ms;
    }
    *count = T.used;
    *mean_ms = T.used ? sum / (double)T.used : 0.0;
    return PSW_OK;
}

psw_status psw_pass_timing(psw_problem *P, double *mean_ms, int64_t *count) {
    if (!P) return PSW_EINVAL;
    return psw_pass_timing_of(P, P->timing_last, mean_ms, count);
}

psw_status psw_autotune(int dim, const int64_t n[3], psw_prec prec, psw_precond kind, int p_out[3],
                        double *us_per_problem, void *stream) {
    if (!n || !p_out || (kind != PSW_SSOR && kind != PSW_ILU0) || prec < PSW_F64 || prec > PSW_BF16) return PSW_EINVAL;
    if (dim != 2) return PSW_ENOTSUP;
    if (n[0] < 2 || n[1] < 2 || n[0] > (1 << 20) || n[1] > (1 << 20)) return PSW_EINVAL;
    int p[2];
    psw_status ps = autotune2d((int)n[0], (int)n[1], prec, kind, p, us_per_problem, (hipStream_t)stream);
    if (ps) return ps;
    p_out[0] = p[0];
    p_out[1] = p[1];
    p_out[2] = 1;
    return PSW_OK;
}

const char *psw_status_string(psw_status st) {
    switch (st) {
    case PSW_OK: return "ok";
    case PSW_EINVAL: return "invalid argument";
    case PSW_ENOMEM: return "out of memory";
    case PSW_EDEVICE: return "HIP error";
    case PSW_ENOCONV: return "not converged";
    case PSW_EBREAKDOWN: return "breakdown";
    case PSW_EPIVOT: return "non-positive ILU pivot";
    case PSW_EBUSY: return "admission refused";
    case PSW_ENOTSUP: return "not supported";
    case PSW_ESTATE: return "call out of order";
    }
    return "unknown status";
}

psw_status psw_problem_create(int dim, const int64_t n[3], int stencil, psw_problem **out) {
    if (!out || !n) return PSW_EINVAL;
    *out = nullptr;
    if (dim < 1 || dim > 3) return PSW_EINVAL;
    if (stencil != 2 * dim + 1) return PSW_EINVAL;
    int64_t N = 1;
    for (int a = 0; a < dim; ++a) {
        if (n[a] < 1 || n[a] > (int64_t)1 << 30) return PSW_EINVAL;
        N *= n[a];
    }
    if (N > ((int64_t)1 << 40)) return PSW_EINVAL;
    psw_problem *P = new (std::nothrow) psw_problem();
    if (!P) return PSW_ENOMEM;
    if (hipGetDevice(&P->device) != hipSuccess) {
        delete P;
        return PSW_EDEVICE;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) == hipSuccess && lds > 0)
        P->lds_limit = (size_t)lds;
    P->dim = dim;
    P->kd = dim < 2 ? 2 : dim;
    for (int a = 0; a < 3; ++a) P->n[a] = a < dim ? (int)n[a] : 1;
    P->N = N;
    *out = P;
    return PSW_OK;
}

psw_status psw_problem_destroy(psw_problem *P) {
    if (!P) return PSW_EINVAL;
    DeviceGuard dg(P->device);
    (void)hipDeviceSynchronize();
    delete P;
    return PSW_OK;
}

// A 1D problem runs on the 2D kernels as an n x 1 grid: its S and N couplings exist and are zero.
static psw_status zero_missing_couplings(psw_problem *P, hipStream_t st) {
    const size_t b = sizeof(double) * (size_t)P->N;
    for (int k = 2 * P->dim + 1; k < 2 * P->kd + 1; ++k) {
        if (!P->diag[k].ensure(b)) return PSW_ENOMEM;
        HIPCHK(hipMemsetAsync(P->diag[k].p, 0, b, st));
    }
    return PSW_OK;
}

// whether the FP64 diagonals are symmetric (checked once, at set-up, on the set-up stream)
static psw_status check_symmetric(psw_problem *P, hipStream_t st) {
    const double *d[7];
    for (int k = 0; k < 7; ++k) d[k] = P->diag[k].as<double>();
    if (!P->symflag.ensure(sizeof(int))) return PSW_ENOMEM;
    int *h = nullptr;
    if (hipHostMalloc((void **)&h, sizeof(int), hipHostMallocDefault) != hipSuccess) return PSW_ENOMEM;
    *h = 1;
    hipError_t e = hipMemcpyAsync(P->symflag.p, h, sizeof(int), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = launch_sym_check(P->kd, P->n, d, P->symflag.as<int>(), st);
    if (e == hipSuccess) e = hipMemcpyAsync(h, P->symflag.p, sizeof(int), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    P->sym = e == hipSuccess && *h == 1;
    (void)hipHostFree(h);
    return e == hipSuccess ? PSW_OK : PSW_EDEVICE;
}

// q = A p in the Krylov loops
static hipError_t krylov_spmv(psw_problem *P, const double *const *d, const double *p, double *q, hipStream_t st) {
    if (P->kd == 3) return launch_spmv3(P->n, d, P->sym, p, q, st);
    return P->sym ? launch_spmv_sym(P->kd, P->n, d, p, q, st) : launch_spmv(P->kd, P->n, d, p, q, st);
}

static void invalidate(psw_problem *P) {
    P->pc[0].ready = false;
    P->pc[1].ready = false;
    P->stat.ready = false;
}

psw_status psw_set_diagonals(psw_problem *P, const double *const diag[], int on_device, psw_prec prec, void *stream) {
    if (!P || !diag || prec < PSW_F64 || prec > PSW_BF16) return PSW_EINVAL;
    psw_status ps;
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    size_t b = sizeof(double) * (size_t)P->N;
    for (int k = 0; k < 2 * P->dim + 1; ++k) {
        if (!diag[k]) return PSW_EINVAL;
        if (!P->diag[k].ensure(b)) return PSW_ENOMEM;
        HIPCHK(hipMemcpyAsync(P->diag[k].p, diag[k], b, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    }
    if ((ps = zero_missing_couplings(P, st))) return ps;
    if ((ps = check_symmetric(P, st))) return ps;
    P->prec = prec;
    P->has_diag = true;
    invalidate(P);
    return PSW_OK;
}

psw_status psw_assemble_diffusion(psw_problem *P, const double *const alpha[], double beta, psw_prec prec,
                                  void *stream) {
    if (!P || !alpha || prec < PSW_F64 || prec > PSW_BF16 || !(beta >= 0.0)) return PSW_EINVAL;
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    size_t b = sizeof(double) * (size_t)P->N;
    double *out[7] = {};
    for (int k = 0; k < 2 * P->dim + 1; ++k) {
        if (!P->diag[k].ensure(b)) return PSW_ENOMEM;
        out[k] = P->diag[k].as<double>();
    }
    for (int a = 0; a < P->dim; ++a)
        if (!alpha[a]) return PSW_EINVAL;
    HIPCHK(launch_assemble(P->dim, P->n, alpha, beta, out, st));
    psw_status ps = zero_missing_couplings(P, st);
    if (ps) return ps;
    if ((ps = check_symmetric(P, st))) return ps;
    P->prec = prec;
    P->has_diag = true;
    invalidate(P);
    return PSW_OK;
}

psw_status psw_get_diagonal(psw_problem *P, int k, double *out, void *stream) {
    if (!P || !out || k < 0 || k > 2 * P->dim) return PSW_EINVAL;
    if (!P->has_diag) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    HIPCHK(hipMemcpyAsync(out, P->diag[k].p, sizeof(double) * P->N, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return PSW_OK;
}

psw_status psw_set_relaxation(psw_problem *P, const double *omega, int count) {
    if (!P || !omega) return PSW_EINVAL;
    int nc = 1 << P->dim;
    if (count != 1 && count != nc) return PSW_EINVAL;
    for (int i = 0; i < count; ++i)
        if (!(omega[i] > 0.0 && omega[i] < 2.0)) return PSW_EINVAL;
    for (int i = 0; i < 8; ++i) P->omega[i] = omega[count == 1 ? 0 : (i < nc ? i : 0)];
    invalidate(P);
    return PSW_OK;
}

psw_status psw_set_decomposition(psw_problem *P, const int p[3], int overlap, int phase) {
    if (!P || !p || overlap < 0 || (phase != 0 && phase != 1)) return PSW_EINVAL;
    int pp[3] = {1, 1, 1};
    for (int a = 0; a < P->dim; ++a) {
        pp[a] = p[a];
        if (pp[a] < 1 || pp[a] > P->n[a]) return PSW_EINVAL;
        if (P->n[a] / pp[a] < 2) return PSW_EINVAL; // every tile at least 2 points long
    }
    DeviceGuard dg(P->device);
    std::vector<int> lo[3], len[3];
    for (int a = 0; a < 3; ++a) partition(P->n[a], pp[a], lo[a], len[a]);
    std::vector<TileDesc> T;
    int cmax = 1, l1max = 1, l2max = 1;
    for (int t = 0; t < pp[2]; ++t)
        for (int s = 0; s < pp[1]; ++s)
            for (int r = 0; r < pp[0]; ++r) {
                TileDesc d{};
                int c[3] = {r, s, t};
                for (int a = 0; a < 3; ++a) {
                    d.lo[a] = lo[a][c[a]];
                    d.len[a] = len[a][c[a]];
                    d.par[a] = c[a] & 1;
                }
                cmax = std::max(cmax, d.len[1] * d.len[2]);
                l1max = std::max(l1max, d.len[1]);
                l2max = std::max(l2max, d.len[2]);
                T.push_back(d);
            }
    if (!P->tiles.ensure(sizeof(TileDesc) * T.size())) return PSW_ENOMEM;
    HIPCHK(hipMemcpy(P->tiles.p, T.data(), sizeof(TileDesc) * T.size(), hipMemcpyHostToDevice));
    P->ntiles = (int)T.size();
    P->cmax = cmax;
    P->l1max = l1max;
    P->l2max = l2max;
    for (int a = 0; a < 3; ++a) P->p[a] = pp[a];
    P->overlap = overlap;
    P->phase = phase;
    P->has_decomp = true;
    invalidate(P);
    return PSW_OK;
}

psw_status psw_precond_apply_noalloc(psw_problem *P, psw_precond kind, const double *r, double *z, void *stream) {
    if (!P || !r || !z || r == z || (kind != PSW_SSOR && kind != PSW_ILU0)) return PSW_EINVAL;
    if ((size_t)P->N * (P->prec == PSW_F64 ? 8 : 4) > kNoAllocScratchBytes) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp || !P->pc[kind].ready) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    void *y = scratch_ptr(P->device);
    if (!y) return PSW_EDEVICE;
    hipStream_t st = (hipStream_t)stream;
    const bool f64 = P->prec == PSW_F64;
    // the forward pass writes every point of y before the backward pass reads it
    psw_status ps = half(P, kind, 0, r, true, false, y, f64, 1.0, st);
    if (ps) return ps;
    return half(P, kind, 1, y, f64, true, z, true, P->pc[kind].c, st);
}

psw_status psw_problem_device_bytes(psw_problem *P, size_t *bytes) {
    if (!P || !bytes) return PSW_EINVAL;
    *bytes = problem_device_bytes(P);
    return PSW_OK;
}

psw_status psw_get_sweep_coefficients(psw_problem *P, psw_precond kind, int k, void *out, void *stream) {
    if (!P || !out || (kind != PSW_SSOR && kind != PSW_ILU0) || k < 0 || k > 2 * P->dim) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    psw_status ps = precond_setup(P, kind, st);
    if (ps) return ps;
    const PrecState &S = P->pc[kind];
    const DevBuf &src = k == 0 ? S.piv : S.diag[k];
    HIPCHK(hipMemcpyAsync(out, src.p, store_bytes(store_of(P->prec)) * (size_t)P->N, hipMemcpyDeviceToDevice, st));
    return PSW_OK;
}

psw_status psw_set_path(psw_problem *P, int path) {
    if (!P || (path != PSW_PATH_AUTO && path != PSW_PATH_GENERIC)) return PSW_EINVAL;
    P->force_generic = path == PSW_PATH_GENERIC;
    invalidate(P);
    return PSW_OK;
}

psw_status psw_sweep(psw_problem *P, int64_t iteration, const double *u_in, const double *f, double *u_out,
                     void *stream) {
    if (!P || !u_in || !f || !u_out || iteration < 0 || u_in == u_out) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    psw_status ps = check_lds(P, 8);
    if (ps) return ps;
    DeviceGuard dg(P->device);
    return sweep_once(P, iteration, u_in, f, u_out, (hipStream_t)stream);
}

psw_status psw_sweep_restricted(psw_problem *P, int64_t iteration, const double *u_in, const double *f,
                                double *u_out, void *stream) {
    if (!P || !u_in || !f || !u_out || iteration < 0 || u_in == u_out) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    return sweep_restricted(P, iteration, u_in, f, u_out, (hipStream_t)stream);
}

psw_status psw_precond_setup(psw_problem *P, psw_precond kind, void *stream) {
    if (!P) return PSW_EINVAL;
    DeviceGuard dg(P->device);
    if (kind == PSW_NONE) return PSW_OK;
    psw_status ps = ensure_work(P);
    if (ps) return ps;
    return precond_setup(P, kind, (hipStream_t)stream);
}

psw_status psw_precond_apply(psw_problem *P, psw_precond kind, int symmetric, const double *r, double *z,
                             void *stream) {
    if (!P || !r || !z || r == z || kind < PSW_SSOR || kind > PSW_NONE) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    return precond_apply(P, kind, symmetric ? 1 : 0, r, z, (hipStream_t)stream);
}

psw_status psw_precond_half(psw_problem *P, psw_precond kind, int which, const double *in, double *out,
                            void *stream) {
    if (!P || !in || !out || in == out || (kind != PSW_SSOR && kind != PSW_ILU0) || which < 0 || which > 3)
        return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    psw_status ps = precond_setup(P, kind, st);
    if (ps) return ps;
    if ((ps = ensure_work(P))) return ps;
    double c = P->pc[kind].c;
    bool scale = (which == 1 || which == 3);
    if (which == 3) {
        if ((ps = half(P, kind, 3, in, true, true, out, true, 1.0, st))) return ps;
        HIPCHK(launch_copy_scaled(out, out, c, P->N, st));
        return PSW_OK;
    }
    return half(P, kind, which, in, true, scale, out, true, which == 1 ? c : 1.0, st);
}

psw_status psw_ilu_pivots(psw_problem *P, double *piv, void *stream) {
    if (!P || !piv) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    psw_status ps = ensure_work(P);
    if (ps) return ps;
    if ((ps = precond_setup(P, PSW_ILU0, st))) return ps;
    HIPCHK(hipMemcpyAsync(piv, P->pc[PSW_ILU0].piv64.p, sizeof(double) * P->N, hipMemcpyDeviceToDevice, st));
    return PSW_OK;
}

psw_status psw_spmv(psw_problem *P, const double *x, double *y, void *stream) {
    if (!P || !x || !y || x == y) return PSW_EINVAL;
    if (!P->has_diag) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    const double *d[7];
    HIPCHK(launch_spmv(P->kd, P->n, diag64(P, d), x, y, (hipStream_t)stream));
    return PSW_OK;
}

psw_status psw_dot(psw_problem *P, const double *x, const double *y, double *out, void *stream) {
    if (!P || !x || !y || !out) return PSW_EINVAL;
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    psw_status ps = ensure_work(P);
    if (ps) return ps;
    double *s = P->scal.as<double>();
    HIPCHK(launch_dot(x, y, P->N, P->partials.as<double>(), s + 11, st));
    HIPCHK(hipMemcpyAsync(out, s + 11, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return PSW_OK;
}

psw_status psw_solve(psw_problem *P, psw_method method, psw_precond precond, double rtol, int64_t maxit, int restart,
                     const double *f, double *u, psw_info *info, void *stream) {
    if (!P || !f || !u || f == u || !(rtol > 0.0) || maxit < 1) return PSW_EINVAL;
    if (precond < PSW_SSOR || precond > PSW_NONE) return PSW_EINVAL;
    if (!P->has_diag || !P->has_decomp) return PSW_ESTATE;
    DeviceGuard dg(P->device);
    hipStream_t st = (hipStream_t)stream;
    double t0 = now_ms();
    psw_info loc{};
    psw_status ps;
    switch (method) {
    case PSW_SOR_STATIONARY: ps = solve_stationary(P, rtol, maxit, f, u, &loc, st); break;
    case PSW_SOR_RESTRICTED: ps = solve_stationary(P, rtol, maxit, f, u, &loc, st, true); break;
    case PSW_CG:
        // a single problem runs on the host-driven loop (psw_batch_solve with count = 1 takes the
        // graph-replayed batch path)
        ps = solve_cg(P, precond, rtol, maxit, f, u, &loc, st);
        break;
    case PSW_FGMRES: ps = solve_fgmres(P, precond, rtol, maxit, restart, f, u, &loc, st); break;
    default: return PSW_EINVAL;
    }
    (void)hipStreamSynchronize(st);
    loc.t_total_ms = now_ms() - t0;
    loc.status = ps;
    if (info) *info = loc;
    return ps;
}

psw_status psw_batch_solve(int count, psw_problem *const *probs, const double *const *f, double *const *u,
                           psw_method method, psw_precond precond, double rtol, int64_t maxit, psw_info *infos,
                           void *stream) {
    if (count < 0 || (count > 0 && (!probs || !f || !u)) || !(rtol > 0.0) || maxit < 1) return PSW_EINVAL;
    if (count == 0) return PSW_OK;
    for (int i = 0; i < count; ++i)
        if (!probs[i] || !f[i] || !u[i] || f[i] == u[i]) return PSW_EINVAL;
    DeviceGuard dg(probs[0]->device);
    bool batched = method == PSW_CG;
    for (int i = 0; i < count && batched; ++i)
        batched = probs[i]->device == probs[0]->device && batch_eligible(probs[i], precond);
    if (batched) {
        psw_status s = batch_cg(count, probs, f, u, precond, rtol, maxit, infos, (hipStream_t)stream);
        if (s != PSW_ENOTSUP) return s;
    }
    psw_status worst = PSW_OK;
    for (int i = 0; i < count; ++i) {
        psw_info inf{};
        psw_status s = psw_solve(probs[i], method, precond, rtol, maxit, 30, f[i], u[i], &inf, stream);
        if (infos) infos[i] = inf;
        if (s != PSW_OK && worst == PSW_OK) worst = s;
    }
    return worst;
}

} // extern "C"
