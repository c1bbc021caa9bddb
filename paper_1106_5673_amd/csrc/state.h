// Device-resident scalar state of the multi-shift CG and the FP64 recurrences
// that update it (Sec. 4.3: the shifted systems (A + sigma_i) x_i = b of
// Eq. shifted are solved from the Krylov space of the smallest shift, with the
// shifted residuals kept collinear with the base one, r_i = zeta_i r).
//
// The recurrences run inside the last workgroup of the kernel that produces
// the reduction they need, so a CG iteration needs no host round trip and can
// be replayed from a hipGraph.
#pragma once

#include "common.h"

namespace rhmc {

struct SysScalars {
    double rr;          // <r, r> of the current residual
    double alpha, alpha_prev, beta_prev;
    double pAp;
    double bnorm;       // ||b|| (FP64)
    double tolb;        // tol * ||b||
    int done;           // every shift of this system met its tolerance (or maxiter)
    int iters;          // iterations completed by this system
    int base;           // index of the shift with offset 0
    int blk_steps;      // iterations this system completed in the current block
};

// Shifted solutions are not touched every iteration.  Between two block
// boundaries k0 and k0+q the recurrences x_i += a_i p_i, p_i = z_i r + b_i p_i
// are carried as coefficients on P = p_i(k0), X = x_i(k0) and the stored base
// residuals r(k0+1..k0+q):
//   p_i(k0+q) = c P + sum_l d[l] r(k0+l)
//   x_i(k0+q) = X + e P + sum_l f[l] r(k0+l)
struct ShiftScalars {
    double off;                 // sigma_i - sigma_0 >= 0
    double zeta, zeta_prev, zeta_next;
    double a;                   // alpha_i of the current step
    double c, e;
    double d[kMaxBlockLen + 1];
    double f[kMaxBlockLen + 1];
    int active;                 // still iterating
    int block_active;           // active when the current block started
    int conv_iter;
    int pad;
};

struct SolverState {
    int nsys, nshift;
    int blk_it;        // iterations completed inside the current block
    int all_done;
    int first_block;   // P = r(k0) and X = 0 (nothing stored yet)
    int iter;          // iterations completed by the shared solve
    int maxiter;
    int reliable_count;
    SysScalars sys[kMaxSys];
    ShiftScalars sh[kMaxSys][kMaxShift];
};

enum FinalizeKind {
    kFinNone = 0,
    kFinInit = 1,      // after the start kernel: ||b||, rr
    kFinAlpha = 2,     // after A p: alpha, zeta_next, a_i
    kFinBeta = 3,      // after r -= alpha A p: beta, b_i, block coefficients, convergence
    kFinReliable = 4,  // after r = b - A x in FP64: rr
    kFinNorms = 5      // plain per-rhs sums into an output array
};

#if defined(__HIPCC__)

// Sum partial[r*nblk + 0..nblk-1] over all threads of the block, fixed order.
__device__ inline double block_sum_partials(const double* partial, int r, int nblk,
                                            double* smem) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partial[(size_t)r * nblk + b];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) smem[wid] = s;
    __syncthreads();
    double t = 0.0;
    const int nw = blockDim.x >> 6;
    for (int w = 0; w < nw; ++w) t += smem[w];
    __syncthreads();
    return t;
}

// Runs in the last block of a reducing kernel (all its threads).
__device__ inline void solver_finalize(int kind, void* vstate, const double* partial, int nblk,
                                       int nrhs, double* out_sums) {
    __shared__ double smem[16];
    __shared__ double sums[2 * kMaxSys];
    if (kind == kFinNorms) {
        for (int r = 0; r < nrhs; ++r) {
            const double t = block_sum_partials(partial, r, nblk, smem);
            if (threadIdx.x == 0) out_sums[r] = t;
        }
        return;
    }
    SolverState* st = reinterpret_cast<SolverState*>(vstate);
    const int nsys = st->nsys;
    const int nsh = st->nshift;
    const int nsum = (kind == kFinInit) ? 2 * nsys : nsys;
    for (int r = 0; r < nsum; ++r) {
        const double t = block_sum_partials(partial, r, nblk, smem);
        if (threadIdx.x == 0) sums[r] = t;
    }
    __syncthreads();
    const int tid = threadIdx.x;

    if (kind == kFinInit) {
        if (tid < nsys) {
            SysScalars& s = st->sys[tid];
            const double b2 = sums[tid];
            s.bnorm = sqrt(b2);
            s.tolb = s.tolb * s.bnorm;   // tolb held the relative tolerance until now
            s.rr = sums[nsys + tid];
            s.alpha = 0.0;
            s.alpha_prev = 1.0;
            s.beta_prev = 0.0;
            s.iters = 0;
            if (!(b2 > 0.0) || !isfinite(b2)) s.done = 1;   // zero or non-finite source
        }
        __syncthreads();
        if (tid == 0) {
            int all = 1;
            for (int j = 0; j < nsys; ++j) all &= st->sys[j].done;
            st->all_done = all;
        }
        return;
    }

    if (kind == kFinReliable) {
        if (tid < nsys && !st->sys[tid].done) st->sys[tid].rr = sums[tid];
        if (tid == 0) st->reliable_count += 1;
        return;
    }

    if (kind == kFinAlpha) {
        if (tid < nsys) {
            SysScalars& s = st->sys[tid];
            if (!s.done) {
                s.pAp = sums[tid];
                s.alpha = s.rr / s.pAp;
            }
        }
        __syncthreads();
        for (int p = tid; p < nsys * nsh; p += blockDim.x) {
            const int j = p / nsh, i = p % nsh;
            const SysScalars s = st->sys[j];
            ShiftScalars* hp = &st->sh[j][i];
            if (s.done || !hp->active) continue;
            const double zeta = hp->zeta, zeta_prev = hp->zeta_prev, off = hp->off;
            const double a = s.alpha;
            const double zn = zeta * zeta_prev * s.alpha_prev /
                              (zeta_prev * s.alpha_prev * (1.0 + a * off) +
                               a * s.beta_prev * (zeta_prev - zeta));
            hp->zeta_next = zn;
            hp->a = a * zn / zeta;
        }
        return;
    }

    // kFinBeta
    __shared__ double beta_s[kMaxSys];
    __shared__ int alive_s[kMaxSys];
    if (tid < nsys) {
        SysScalars& s = st->sys[tid];
        beta_s[tid] = s.done ? 0.0 : sums[tid] / s.rr;
        alive_s[tid] = 0;
    }
    __syncthreads();
    const int q_all = st->blk_it;
    for (int p = tid; p < nsys * nsh; p += blockDim.x) {
        const int j = p / nsh, i = p % nsh;
        const SysScalars s = st->sys[j];
        ShiftScalars* hp = &st->sh[j][i];
        if (s.done || !hp->active) continue;
        // one bulk copy into registers, update, one bulk copy back
        ShiftScalars h = *hp;
        const int q = s.blk_steps;   // this step's index inside the block (0-based)
        const double ratio = h.zeta_next / h.zeta;
        const double bi = beta_s[j] * ratio * ratio;
        // x_i(k+1) = x_i(k) + a_i p_i(k);  p_i(k) = c P + sum_{l<=q} d[l] r(k0+l)
        h.e += h.a * h.c;
        // p_i(k+1) = zeta_i(k+1) r(k+1) + b_i p_i(k)
        h.c *= bi;
        // (fully unrolled with compile-time indices so h stays in registers)
#pragma unroll
        for (int l = 1; l <= kMaxBlockLen; ++l) {
            if (l <= q) {
                h.f[l] += h.a * h.d[l];
                h.d[l] *= bi;
            } else if (l == q + 1) {
                h.d[l] = h.zeta_next;
            }
        }
        h.zeta_prev = h.zeta;
        h.zeta = h.zeta_next;
        const double res = fabs(h.zeta) * sqrt(sums[j]);
        if (res <= s.tolb) {
            h.active = 0;
            h.conv_iter = s.iters + 1;
        }
        *hp = h;
    }
    __syncthreads();
    for (int p = tid; p < nsys * nsh; p += blockDim.x) {
        const int j = p / nsh, i = p % nsh;
        if (st->sh[j][i].active) atomicOr(&alive_s[j], 1);
    }
    __syncthreads();
    if (tid < nsys) {
        SysScalars& s = st->sys[tid];
        if (!s.done) {
            s.alpha_prev = s.alpha;
            s.beta_prev = beta_s[tid];
            s.rr = sums[tid];
            s.iters += 1;
            s.blk_steps += 1;
            if (!alive_s[tid] || s.iters >= st->maxiter || !isfinite(s.rr)) s.done = 1;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int all = 1;
        for (int j = 0; j < nsys; ++j) all &= st->sys[j].done;
        st->all_done = all;
        st->blk_it = q_all + 1;
        st->iter += 1;
    }
}

#endif  // __HIPCC__

}  // namespace rhmc
