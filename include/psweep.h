/*
 * psweep.h -- C ABI of libpsweep.so: parallel SOR / SSOR / ILU(0) sweeps on
 * structured 5-point (2D) and 7-point (3D) n-diagonal matrices, made parallel
 * by the overlapping block decomposition and multi-frontal sweep ordering of
 * R. Tavakoli, "Parallelizing sequential sweeping on structured grids --
 * fully parallel SOR/ILU preconditioners for structured n-diagonal matrices".
 * The kernels are HIP for gfx950 (MI355X).
 *
 * Problem statement (Sec. 7): solve or precondition A u = f where A is an
 * irreducibly diagonally dominant structured n-diagonal matrix on a
 * structured grid.
 *
 * Layout.  dim in {1,2,3}; n[a] interior points on axis a; point index
 * P = x + n0*(y + n1*z) (x fastest).  Boundary points are not stored:
 * Dirichlet data are folded into f (eq. 1d:mat, eq. d2d).  Diagonals come in
 * the order P, W, E, S, N, B, F (2*dim+1 arrays of N doubles; W/E = -x/+x,
 * S/N = -y/+y, B/F = -z/+z) with the sign convention of eq. d2d:
 *     a^P_P u_P - sum_X a^X_P u_{P+e_X} = f_P ,   a^X >= 0 expected.
 * Couplings that point outside the grid are ignored.
 *
 * Pointers.  Every vector argument is a device pointer (HIP global memory,
 * e.g. a torch tensor's data_ptr()) of N doubles unless stated otherwise; the
 * caller owns it.  The library never keeps or frees a caller pointer; it
 * copies diagonals into its own device arrays.  `stream` is a hipStream_t
 * (NULL = the default stream); every call is ordered on that stream and
 * returns after enqueueing unless it says otherwise.
 *
 * Errors.  Every call returns a psw_status and never throws.  A handle is not
 * thread-safe; the server object is.
 */
#ifndef PSWEEP_H
#define PSWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PSW_OK = 0,
    PSW_EINVAL = -1,     /* bad argument (dims, sizes, omega, partition, pointer) */
    PSW_ENOMEM = -2,     /* device or host allocation failed */
    PSW_EDEVICE = -3,    /* a HIP call failed */
    PSW_ENOCONV = -4,    /* iteration limit reached before the tolerance */
    PSW_EBREAKDOWN = -5, /* Krylov breakdown (p.Ap <= 0, zero Arnoldi norm, NaN/Inf residual) */
    PSW_EPIVOT = -6,     /* non-positive ILU(0) pivot */
    PSW_EBUSY = -7,      /* admission refused: memory budget exhausted */
    PSW_ENOTSUP = -8,    /* combination not supported by this build */
    PSW_ESTATE = -9      /* call out of order (e.g. sweep before diagonals are set) */
} psw_status;

/* precision of the preconditioner sweeps: FP64; FP32 diagonals and FP32
   arithmetic; BF16-stored diagonals with FP32 arithmetic.  Outer vectors,
   residuals, dot products and updates are always FP64. */
typedef enum { PSW_F64 = 0, PSW_F32 = 1, PSW_BF16 = 2 } psw_prec;
typedef enum { PSW_SSOR = 0, PSW_ILU0 = 1, PSW_NONE = 2 } psw_precond;
typedef enum { PSW_SOR_STATIONARY = 0, PSW_CG = 1, PSW_FGMRES = 2, PSW_SOR_RESTRICTED = 3 } psw_method;

typedef struct psw_problem psw_problem;

typedef struct {
    int64_t iters;       /* sweeps (stationary) or Krylov iterations */
    double relres;       /* final ||f - A u||_2 / ||f||_2, recomputed at exit */
    int converged;       /* 1 if relres <= rtol was reached */
    int status;          /* psw_status of the solve */
    double t_total_ms;   /* wall time of the solve on the host clock */
    double t_precond_ms; /* time in preconditioner kernels (HIP events; 0 if not measured) */
} psw_info;

/* Create a problem on a dim-dimensional grid with n[0..dim-1] interior
 * points; stencil must be 2*dim+1 (3, 5 or 7).  A 1D (tridiagonal) problem
 * (Sec. 2) runs on the 2D kernels as an n x 1 grid; its schedule is the 1D
 * one (+ then -), its coupled blocks the 2x2 of eq. 1d:sorc.  Memory for the handle is owned
 * by the library; free it with psw_problem_destroy.  The current HIP device
 * at creation is used for every later call on the handle. */
psw_status psw_problem_create(int dim, const int64_t n[3], int stencil, psw_problem **out);
psw_status psw_problem_destroy(psw_problem *prob);

/* Set the matrix from 2*dim+1 diagonal arrays (order P,W,E,S,N,B,F), host
 * (on_device=0) or device (on_device=1) pointers.  sweep_prec selects the
 * precision of the preconditioner sweeps.  Invalidates preconditioner state. */
psw_status psw_set_diagonals(psw_problem *prob, const double *const diag[], int on_device,
                             psw_prec sweep_prec, void *stream);

/* Assemble the diagonals of -div(alpha grad u) + beta u on a unit-spaced
 * grid (eq. d2d; Sec. 3 harmonic face means) on the device.  alpha[a],
 * a < dim, is the axis-a coefficient on all (n0+2)*(n1+2)[*(n2+2)] nodes,
 * boundary ring included, node (i,j,k) at i + (n0+2)*(j + (n1+2)*k) and
 * interior point x at node x+1.  Face coupling = harmonic mean of the two
 * node values; a^P = sum of the 2*dim face couplings + beta.  Device
 * pointers.  Equivalent to psw_set_diagonals with the assembled arrays. */
psw_status psw_assemble_diffusion(psw_problem *prob, const double *const alpha[], double beta,
                                  psw_prec sweep_prec, void *stream);

/* Copy diagonal k (0 = P ... 2*dim) into the device array out (N doubles). */
psw_status psw_get_diagonal(psw_problem *prob, int k, double *out, void *stream);

/* Relaxation factors per start corner (Sec. 3: omega_SW, omega_NE, ...): count = 1
 * (same factor everywhere) or 2^dim, indexed by the start corner of the
 * sweep: bit a set when the sweep along axis a starts at the high end (so in
 * 2D: 0 = SW, 1 = SE, 2 = NW, 3 = NE).  Each factor must lie in (0,2).
 * The SSOR preconditioner uses omega[0]. */
psw_status psw_set_relaxation(psw_problem *prob, const double *omega, int count);

/* Decomposition into p[0] x p[1] (x p[2]) subdomains: contiguous ranges per
 * axis, the first n mod p ranges one point longer (Sec. 3).  Every
 * subdomain must be at least 2 points long on every axis.  overlap (>= 0) is
 * the number of points by which the restricted-overlap sweep
 * (psw_sweep_restricted) widens every subdomain's box.  The exact-coupling
 * sweep, its preconditioners and solves read one layer beyond a subdomain
 * (two across a coupled start face, Sec. 3, Data structure) whatever the
 * overlap, so their results do not depend on it.  phase swaps the two
 * members of every direction pair of the schedule (Sec. 3, Sweeping
 * directions). */
psw_status psw_set_decomposition(psw_problem *prob, const int p[3], int overlap, int phase);

/* Kernel path of the preconditioner passes: PSW_PATH_AUTO (the pipelined 2D
 * passes and the 3D LDS-tile passes where a decomposition fits them) or
 * PSW_PATH_GENERIC (the level-by-level kernels for every pass).  Both compute
 * the same operator; the switch exists so that tests and measurements can
 * compare the two.  Invalidates preconditioner state. */
enum { PSW_PATH_AUTO = 0, PSW_PATH_GENERIC = 1 };
psw_status psw_set_path(psw_problem *prob, int path);

/* One decomposed SOR sweep, FP64 (Secs. 2-4).  Subdomain (r,s,t) sweeps at
 * iteration k in direction sigma_{k mod 2^dim} with the sign of axis a
 * flipped for odd coordinate a; base cycle 2D: (-,-),(+,+),(+,-),(-,+);
 * 3D: (-,-,-),(+,+,+),(+,-,-),(-,+,+),(-,+,-),(+,-,+),(+,+,-),(-,-,+).
 * Every point takes new values from the neighbours on the side where its own
 * subdomain's sweep begins and old values from u_in on the other side;
 * points of start faces shared with a neighbour that also starts there are
 * solved jointly with their partners (eq. 2d:sor2b2, 2x2; eq. 2d:sor4b4,
 * 4x4; the 3D 4x4 and 8x8 systems of Sec. 4).  u_in, f, u_out are device
 * arrays of N doubles; u_out must not alias u_in. */
psw_status psw_sweep(psw_problem *prob, int64_t iteration, const double *u_in, const double *f,
                     double *u_out, void *stream);

/* One restricted-overlap sweep, FP64: the reading of the paper's parallel
 * experiments under which its PGS/PSOR iteration counts (Sec. 8, Tables
 * 1d:1-3d:3) are reproduced, in place of the exact coupled blocks of
 * psw_sweep.  Subdomain s, with the direction of psw_sweep's schedule at
 * this iteration, widens its box by the decomposition's overlap on every
 * side (clipped to the grid), sweeps the widened box lexicographically in its
 * direction with the relaxation factor of its start corner, taking u_in
 * outside the widened box, and writes only its own points to u_out.  With
 * overlap 1 the paper's PGS/PSOR counts are matched within 2 %.  PSW_ENOTSUP
 * when the widened box of the largest subdomain with a ring of one point
 * (FP64) exceeds one workgroup's LDS.  Device arrays; u_out must not alias
 * u_in.  psw_solve with PSW_SOR_RESTRICTED iterates it to a tolerance. */
psw_status psw_sweep_restricted(psw_problem *prob, int64_t iteration, const double *u_in, const double *f,
                                double *u_out, void *stream);

/* Build the preconditioner state (pivots, packed diagonals) for kind.  Done
 * implicitly by the first psw_precond_apply / psw_solve; returns PSW_EPIVOT
 * if an ILU(0) pivot is not positive.  The preconditioner uses the direction
 * map of schedule step 0 (d) for its forward half-sweep and -d for its
 * backward half-sweep (Sec. 5: a symmetric Gauss-Seidel pass of the parallel
 * sweep is the parallel ILU(0) / SSOR preconditioner). */
psw_status psw_precond_setup(psw_problem *prob, psw_precond kind, void *stream);

/* z = M^-1 r (symmetric = 0) or z = (M^-1 + M^-T) r / 2 (symmetric = 1) with
 *   SSOR : M^-1 = (2-w) (D/w - N2)^-1 (D/w) (D/w - N1)^-1
 *   ILU0 : M^-1 = (D~ - N2)^-1 D~ (D~ - N1)^-1
 * N1 / N2: upstream couplings under d / -d (N1 + N2 = all off-diagonal
 * couplings); D~: ILU(0) pivots of the decomposed factorisation.  r and z
 * are device arrays of N doubles and must not alias.  PSW_NONE copies. */
psw_status psw_precond_apply(psw_problem *prob, psw_precond kind, int symmetric, const double *r,
                             double *z, void *stream);

/* z = M^-1 r (the pair form of psw_precond_apply, symmetric = 0) without
 * allocating: for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid it).  The
 * intermediate vector of the forward pass lives in a fixed 64 MiB device
 * array of the library, one per GPU, held until the process ends; N times
 * the intermediate's element size (8 bytes for FP64 sweeps, 4 for FP32 and
 * BF16) must fit in it, else PSW_EINVAL.  The preconditioner must already be
 * set up (psw_precond_setup or an earlier apply or solve), else PSW_ESTATE.
 * Every call on a GPU uses that GPU's one array: calls that overlap in time on
 * one GPU (other streams, other threads, other handles) race and give wrong
 * results; calls ordered on one stream are safe.  Results are identical to
 * psw_precond_apply with symmetric = 0. */
psw_status psw_precond_apply_noalloc(psw_problem *prob, psw_precond kind, const double *r, double *z,
                                     void *stream);

/* One half-sweep of the preconditioner, FP64 in and out (for measurement and
 * tests): which = 0: y = (Piv - N1)^-1 r;  1: z = c (Piv - N2)^-1 Piv y;
 * 2: y = (Piv - N2)^-T r;  3: z = c (Piv - N1)^-T Piv y.  (Piv, c) =
 * (D/w, 2-w) for SSOR and (D~, 1) for ILU0. */
psw_status psw_precond_half(psw_problem *prob, psw_precond kind, int which, const double *in,
                            double *out, void *stream);

/* The preconditioner's stored coefficients in the sweep precision, as the
 * kernels read them: k = 0 the pivots (D/w for SSOR, D~ for ILU0), k = 1..2*dim
 * the couplings of diagonal k (W,E,S,N,B,F).  out is a device array of N
 * elements of the sweep precision (8, 4 or 2 bytes: FP64, FP32, or BF16, the
 * upper 16 bits of an FP32), each the round-to-nearest-even conversion of the
 * FP64 value of the Sec. 5 forms.  For tests of the conversion; sets the
 * preconditioner up if needed. */
psw_status psw_get_sweep_coefficients(psw_problem *prob, psw_precond kind, int k, void *out, void *stream);

/* Device memory the handle holds now, in bytes (its own arrays; the caller's
 * vectors are not counted). */
psw_status psw_problem_device_bytes(psw_problem *prob, size_t *bytes);

/* ILU(0) pivots D~ of the decomposed factorisation (FP64, N doubles):
 * D~_P = a^P_P - sum_{Q upstream of P in P's subdomain} a_{P->Q} a_{Q->P} / D~_Q. */
psw_status psw_ilu_pivots(psw_problem *prob, double *piv, void *stream);

/* y = A x (device arrays, N doubles, no aliasing). */
psw_status psw_spmv(psw_problem *prob, const double *x, double *y, void *stream);

/* Deterministic dot product x.y (fixed reduction order independent of the
 * launch); result written to *out on the host after the stream drains. */
psw_status psw_dot(psw_problem *prob, const double *x, const double *y, double *out, void *stream);

/* Solve A u = f to ||f - A u||_2 / ||f||_2 <= rtol from the initial guess in
 * u.  method: stationary decomposed SOR (precond ignored; PSW_SOR_RESTRICTED
 * iterates psw_sweep_restricted instead of psw_sweep), CG with the
 * symmetric form (M^-1 + M^-T)/2 of the preconditioner, or right-
 * preconditioned flexible GMRES(restart) with M^-1.  Returns PSW_ENOCONV when
 * maxit is reached.  info may be NULL.  Blocks until the solve ends. */
psw_status psw_solve(psw_problem *prob, psw_method method, psw_precond precond, double rtol,
                     int64_t maxit, int restart, const double *f, double *u, psw_info *info,
                     void *stream);

/* Solve count independent problems (each with its own handle, decomposition
 * and preconditioner) with CG and the symmetric preconditioner, interleaving
 * their iterations so that the device works on all of them at once.
 * Converged problems drop out.  infos[i] receives each result. */
psw_status psw_batch_solve(int count, psw_problem *const *probs, const double *const *f,
                           double *const *u, psw_method method, psw_precond precond, double rtol,
                           int64_t maxit, psw_info *infos, void *stream);

/* Autotuner for batched solves: choose subdomain counts p_out for a 2D
 * problem of n[0] x n[1] points by timing candidate tile sides (16 to 128
 * points) on the batched symmetric preconditioner, with the problem
 * replicated until its tiles fill the device; the cheapest per problem wins.
 * The choice changes speed only: with exact coupled blocks the
 * preconditioner quality barely depends on the tile size.  Results are
 * cached per (size, precision, preconditioner) for the life of the process.
 * us_per_problem (may be NULL) receives the winning time per problem and
 * preconditioner application, or -1 when the answer came from the cache.
 * PSW_ENOTSUP for 3D. */
psw_status psw_autotune(int dim, const int64_t n[3], psw_prec prec, psw_precond kind, int p_out[3],
                        double *us_per_problem, void *stream);

/* Measurement aid: while enabled, the library records HIP events on the
 * launching stream around every 8th launch (at most 1024) of pipelined pass
 * `which` (0..3; the 2D pipelined path only) of this problem, inside solves
 * and preconditioner calls alike; which = 4 selects the fused step of 2D CG
 * (p update, q = A p and the p.q partials).  psw_pass_timing returns the mean duration
 * of the recorded launches in ms and their number since the last enable
 * (it waits for them to complete) for the pass enabled last.  Enabling resets that pass's record. */
psw_status psw_pass_timing_enable(psw_problem *prob, int which, int enable);
psw_status psw_pass_timing(psw_problem *prob, double *mean_ms, int64_t *count);
/* The same for pass `which` (0..4); each pass keeps its own record, so several
 * can be timed in the same solves. */
psw_status psw_pass_timing_of(psw_problem *prob, int which, double *mean_ms, int64_t *count);

/* ---------------------------------------------------------------- serving
 * A server solves a stream of independent problems A u = f with
 * -div(alpha grad u) + beta u on unit-spaced grids (2D 5-point or 3D
 * 7-point), CG with the symmetric form of the preconditioner, u0 = 0.
 * Admission reserves an estimate of each request's device memory against
 * budget_bytes; requests wait in arrival order until their reservation fits.
 * 2D requests are batched continuously: between epochs of epoch_iters CG
 * iterations of all active 2D problems, admitted requests join and finished
 * ones leave and free their memory.  3D requests are solved by lanes3d worker
 * lanes, one request each at a time on its own stream, overlapping with the
 * 2D batch and with each other.  A request's arithmetic
 * does not depend on the other requests in the batch.  Thread-safe. */
typedef struct psw_server psw_server;
typedef struct {
    psw_prec prec;       /* sweep precision (outer CG is FP64) */
    psw_precond precond; /* PSW_SSOR (omega = 1) or PSW_ILU0 */
    double rtol;         /* relative residual tolerance */
    int64_t maxit;       /* iteration limit per request */
    int epoch_iters;     /* CG iterations between admissions (rounded up to even; <= 0: 16) */
    int max_active;      /* most 2D problems in the batch at once (<= 0: 1024) */
    int lanes3d;         /* 3D requests solved at once, each on its own stream (<= 0: 4; at most 16) */
} psw_server_opts;

psw_status psw_server_create(size_t budget_bytes, const psw_server_opts *opts, psw_server **out);
/* Queue a request.  alpha[a] (a < dim): axis-a coefficients on the (n+2)^dim
 * nodes, as in psw_assemble_diffusion; f: N right-hand-side values; host
 * arrays, copied before return.  PSW_EBUSY if the request alone exceeds the
 * budget.  *ticket identifies the request. */
psw_status psw_server_submit(psw_server *srv, int dim, const int64_t n[3], const double *const alpha[], double beta,
                             const double *f, uint64_t *ticket);
/* The device bytes admission reserves for a request of this shape: the
 * footprint of its problem (diagonals, workspace, the preconditioner's
 * packings for the largest of the decompositions the autotuner may choose),
 * its right-hand side and solution, and its node coefficients during set-up. */
psw_status psw_server_request_bytes(psw_server *srv, int dim, const int64_t n[3], size_t *bytes);

/* *done = 1 once the request has finished (wait = 1 blocks until then).  On
 * completion info receives iterations, relres, status and t_total_ms =
 * submission to completion; t_queue_ms (may be NULL) the time spent waiting
 * for admission; u (host, N doubles, may be NULL) the solution.  A finished
 * request is returned once; its ticket is then forgotten. */
psw_status psw_server_poll(psw_server *srv, uint64_t ticket, int wait, int *done, psw_info *info, double *u,
                           double *t_queue_ms);
/* Finish every queued request, then stop the workers and free the server. */
psw_status psw_server_destroy(psw_server *srv);

/* Readable name of a status code (static storage). */
const char *psw_status_string(psw_status st);

#ifdef __cplusplus
}
#endif

#endif /* PSWEEP_H */
