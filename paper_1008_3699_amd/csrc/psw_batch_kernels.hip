// psw_batch_kernels.hip -- FP64 vector kernels over a batch of problems.
//
// A batch is a table of problems (BProb: pointers to each problem's own
// vectors and scalars) and a table of vector chunks, each inside one problem.
// One launch covers every chunk of every active problem.  Reductions are
// formed per chunk in a fixed order and then per problem over its own chunks
// in chunk order, so a problem's dot products -- and therefore its whole
// iteration -- are bitwise the same whether it is solved alone or in a batch.
#include "psw_batch.h"

#include <hip/hip_runtime.h>

namespace psw {

namespace {

constexpr int kT = 256;

__device__ __forceinline__ double *vslot(const BProb &P, int k) { return reinterpret_cast<double *>(P.vec[k]); }

__device__ __forceinline__ double block_sum256(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// y = A x (or y = f - A x when residual); blocks walk the chunks
__global__ void __launch_bounds__(kT) k_b_spmv(const BChunk *chunks, int nc, const BProb *probs, int src, int dst,
                                              int residual) {
    for (int ci = blockIdx.x; ci < nc; ci += gridDim.x) {
        const BChunk c = chunks[ci];
        const BProb &P = probs[c.prob];
        if (P.flags[0] == 0) continue;
        const double *__restrict__ x = vslot(P, src);
        double *__restrict__ y = vslot(P, dst);
        const double *__restrict__ f = vslot(P, kSlotF);
        const double *__restrict__ d0 = P.diag64[0], *__restrict__ d1 = P.diag64[1], *__restrict__ d2 = P.diag64[2];
        const double *__restrict__ d3 = P.diag64[3], *__restrict__ d4 = P.diag64[4];
        const int n0 = P.n0, n1 = P.n1;
        const int start = (int)c.start;
        for (int k = threadIdx.x; k < c.len; k += kT) {
            const int i = start + k;
            const int iy = i / n0, ix = i - iy * n0;
            double acc = d0[i] * x[i];
            if (ix > 0) acc -= d1[i] * x[i - 1];
            if (ix < n0 - 1) acc -= d2[i] * x[i + 1];
            if (iy > 0) acc -= d3[i] * x[i - n0];
            if (iy < n1 - 1) acc -= d4[i] * x[i + n0];
            y[i] = residual ? f[i] - acc : acc;
        }
    }
}

__global__ void __launch_bounds__(kT) k_b_dot_partial(const BChunk *chunks, int nc, const BProb *probs, int a, int b,
                                                     double *partials) {
    __shared__ double sh[kT];
    for (int ci = blockIdx.x; ci < nc; ci += gridDim.x) {
        const BChunk c = chunks[ci];
        const BProb &P = probs[c.prob];
        if (P.flags[0] == 0) continue; // uniform per block
        const double *__restrict__ x = vslot(P, a), *__restrict__ y = vslot(P, b);
        const int start = (int)c.start;
        double acc = 0.0;
        for (int k = threadIdx.x; k < c.len; k += kT) acc += x[start + k] * y[start + k];
        const double s = block_sum256(acc, sh);
        if (threadIdx.x == 0) partials[ci] = s;
        __syncthreads();
    }
}

// one block per problem: its chunk partials, strided over the threads in a
// fixed order and then summed by a fixed tree
__global__ void __launch_bounds__(kT) k_b_dot_final(const BProb *probs, int nprob, const double *partials, int dst,
                                                   int force) {
    __shared__ double sh[kT];
    const int b = blockIdx.x;
    if (b >= nprob) return;
    const BProb &P = probs[b];
    if (P.flags[0] == 0 && !force) return;
    double acc = 0.0;
    for (int k = threadIdx.x; k < P.nchunk; k += kT) acc += partials[P.chunk0 + k];
    const double s = block_sum256(acc, sh);
    if (threadIdx.x == 0) P.scal[dst] = s;
}

// x += alpha p, r -= alpha q with alpha = scal[num] / scal[2]; partial r.r
__global__ void __launch_bounds__(kT) k_b_cg_xr(const BChunk *chunks, int nc, const BProb *probs, int num,
                                               double *partials) {
    __shared__ double sh[kT];
    for (int ci = blockIdx.x; ci < nc; ci += gridDim.x) {
        const BChunk c = chunks[ci];
        const BProb &P = probs[c.prob];
        if (P.flags[0] == 0) continue;
        const double alpha = P.scal[num] / P.scal[2];
        double *__restrict__ x = vslot(P, kSlotX), *__restrict__ r = vslot(P, kSlotR);
        const double *__restrict__ p = vslot(P, kSlotP), *__restrict__ q = vslot(P, kSlotQ);
        const int start = (int)c.start;
        double acc = 0.0;
        for (int k = threadIdx.x; k < c.len; k += kT) {
            const int i = start + k;
            x[i] += alpha * p[i];
            const double ri = r[i] - alpha * q[i];
            r[i] = ri;
            acc += ri * ri;
        }
        const double s = block_sum256(acc, sh);
        if (threadIdx.x == 0) partials[ci] = s;
        __syncthreads();
    }
}

// one thread per problem, after an x / r update: count the iteration, stop on
// convergence, iteration limit or breakdown
__global__ void k_b_check(const BProb *probs, int nprob, double rtol2, int64_t maxit) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    const BProb &P = probs[b];
    if (P.flags[0] == 0) return;
    const int it = P.flags[1] + 1;
    P.flags[1] = it;
    const double rr = P.scal[3], pq = P.scal[2];
    if (!(pq > 0.0) || !(rr == rr) || rr > 1e300) {
        P.flags[0] = 0;
        P.flags[2] = -5; // breakdown
    } else if (rr <= rtol2 * P.scal[4]) {
        P.flags[0] = 0;
        P.flags[2] = 0;
    } else if (it >= maxit) {
        P.flags[0] = 0;
        P.flags[2] = -4;
    }
}

// start of a solve: active unless the initial residual already meets the tolerance
__global__ void k_b_init(const BProb *probs, int nprob, double rtol2) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    const BProb &P = probs[b];
    P.flags[1] = 0;
    const bool done = P.scal[3] <= rtol2 * P.scal[4];
    P.flags[0] = done ? 0 : 1;
    P.flags[2] = done ? 0 : -4;
}

__global__ void k_b_activate(const BProb *probs, int nprob) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nprob) probs[b].flags[0] = 1;
}

__global__ void k_b_count(const BProb *probs, int nprob, int *out) {
    __shared__ int sh[kT];
    int acc = 0;
    for (int b = threadIdx.x; b < nprob; b += kT) acc += probs[b].flags[0] ? 1 : 0;
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kT / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = sh[0];
}

// per problem: iflags[3 b + k] = flags[k] (k < 3), dscal[5 b + k] = scal[k] (k < 5)
__global__ void k_b_gather(const BProb *probs, int nprob, int *iflags, double *dscal) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nprob) return;
    const BProb &p = probs[b];
    for (int k = 0; k < 3; ++k) iflags[3 * b + k] = p.flags[k];
    if (dscal)
        for (int k = 0; k < 5; ++k) dscal[5 * b + k] = p.scal[k];
}

// p = z + beta p, beta = scal[num] / scal[den]
__global__ void __launch_bounds__(kT) k_b_cg_p(const BChunk *chunks, int nc, const BProb *probs, int num, int den) {
    for (int ci = blockIdx.x; ci < nc; ci += gridDim.x) {
        const BChunk c = chunks[ci];
        const BProb &P = probs[c.prob];
        if (P.flags[0] == 0) continue;
        const double beta = P.scal[num] / P.scal[den];
        double *__restrict__ p = vslot(P, kSlotP);
        const double *__restrict__ z = vslot(P, kSlotZ);
        const int start = (int)c.start;
        for (int k = threadIdx.x; k < c.len; k += kT) p[start + k] = z[start + k] + beta * p[start + k];
    }
}

// z = (z1 + c x) / 2 with x in the sweep precision (slot y1)
__global__ void __launch_bounds__(kT) k_b_combine(const BChunk *chunks, int nc, const BProb *probs, int y_f64) {
    for (int ci = blockIdx.x; ci < nc; ci += gridDim.x) {
        const BChunk c = chunks[ci];
        const BProb &P = probs[c.prob];
        if (P.flags[0] == 0) continue;
        double *__restrict__ z = vslot(P, kSlotZ);
        const double *__restrict__ z1 = vslot(P, kSlotZ1);
        const double hc = 0.5 * P.c;
        const int start = (int)c.start;
        if (y_f64) {
            const double *__restrict__ y = reinterpret_cast<const double *>(P.vec[kSlotY1]);
            for (int k = threadIdx.x; k < c.len; k += kT) z[start + k] = 0.5 * z1[start + k] + hc * y[start + k];
        } else {
            const float *__restrict__ y = reinterpret_cast<const float *>(P.vec[kSlotY1]);
            for (int k = threadIdx.x; k < c.len; k += kT) z[start + k] = 0.5 * z1[start + k] + hc * (double)y[start + k];
        }
    }
}

__global__ void __launch_bounds__(kT) k_b_copy(const BChunk *chunks, int nc, const BProb *probs, int src, int dst) {
    for (int ci = blockIdx.x; ci < nc; ci += gridDim.x) {
        const BChunk c = chunks[ci];
        const BProb &P = probs[c.prob];
        if (P.flags[0] == 0) continue;
        const double *__restrict__ a = vslot(P, src);
        double *__restrict__ b = vslot(P, dst);
        const int start = (int)c.start;
        for (int k = threadIdx.x; k < c.len; k += kT) b[start + k] = a[start + k];
    }
}

} // namespace

static dim3 cgrid(int nc) { return dim3(nc < 8192 ? nc : 8192); }

hipError_t launch_b_spmv(const BChunk *c, int nc, const BProb *p, int src, int dst, bool residual, hipStream_t st) {
    hipLaunchKernelGGL(k_b_spmv, cgrid(nc), dim3(kT), 0, st, c, nc, p, src, dst, residual ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_b_dot(const BChunk *c, int nc, const BProb *p, int np, int a, int b, double *partials, int dst,
                        bool force, hipStream_t st) {
    hipLaunchKernelGGL(k_b_dot_partial, cgrid(nc), dim3(kT), 0, st, c, nc, p, a, b, partials);
    hipLaunchKernelGGL(k_b_dot_final, dim3(np), dim3(kT), 0, st, p, np, (const double *)partials, dst, force ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_b_cg_xr(const BChunk *c, int nc, const BProb *p, int np, int num, double *partials,
                          hipStream_t st) {
    hipLaunchKernelGGL(k_b_cg_xr, cgrid(nc), dim3(kT), 0, st, c, nc, p, num, partials);
    hipLaunchKernelGGL(k_b_dot_final, dim3(np), dim3(kT), 0, st, p, np, (const double *)partials, 3, 0);
    return hipGetLastError();
}

hipError_t launch_b_check(const BProb *p, int np, double rtol2, int64_t maxit, hipStream_t st) {
    hipLaunchKernelGGL(k_b_check, dim3((np + 63) / 64), dim3(64), 0, st, p, np, rtol2, maxit);
    return hipGetLastError();
}

hipError_t launch_b_init(const BProb *p, int np, double rtol2, hipStream_t st) {
    hipLaunchKernelGGL(k_b_init, dim3((np + 63) / 64), dim3(64), 0, st, p, np, rtol2);
    return hipGetLastError();
}

hipError_t launch_b_activate(const BProb *p, int np, hipStream_t st) {
    hipLaunchKernelGGL(k_b_activate, dim3((np + 63) / 64), dim3(64), 0, st, p, np);
    return hipGetLastError();
}

hipError_t launch_b_count(const BProb *p, int np, int *out, hipStream_t st) {
    hipLaunchKernelGGL(k_b_count, dim3(1), dim3(kT), 0, st, p, np, out);
    return hipGetLastError();
}

hipError_t launch_b_gather(const BProb *p, int np, int *iflags, double *dscal, hipStream_t st) {
    hipLaunchKernelGGL(k_b_gather, dim3((np + 63) / 64), dim3(64), 0, st, p, np, iflags, dscal);
    return hipGetLastError();
}

hipError_t launch_b_cg_p(const BChunk *c, int nc, const BProb *p, int num, int den, hipStream_t st) {
    hipLaunchKernelGGL(k_b_cg_p, cgrid(nc), dim3(kT), 0, st, c, nc, p, num, den);
    return hipGetLastError();
}

hipError_t launch_b_combine(const BChunk *c, int nc, const BProb *p, bool y_f64, hipStream_t st) {
    hipLaunchKernelGGL(k_b_combine, cgrid(nc), dim3(kT), 0, st, c, nc, p, y_f64 ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_b_copy(const BChunk *c, int nc, const BProb *p, int src, int dst, hipStream_t st) {
    hipLaunchKernelGGL(k_b_copy, cgrid(nc), dim3(kT), 0, st, c, nc, p, src, dst);
    return hipGetLastError();
}

} // namespace psw
