// Device-resident scalar state of the multi-shift CG and the FP64 recurrences
// that update it (Sec. 4.3: the shifted systems (A + sigma_i) x_i = b of
// Eq. shifted are solved from the Krylov space of the smallest shift, with the
// shifted residuals kept collinear with the base one, r_i = zeta_i r).
//
// No host round trip is needed inside the iteration loop: every kernel reads
// the scalars it needs from device memory, and one block updates them, so a
// block of iterations can be replayed from a hipGraph.
#pragma once

#include "common.h"

namespace rhmc {

struct SysScalars {
    double rr[2];       // <r, r>, double-buffered by step parity (see iteration_update)
    double pap;         // <p, A p> of the current step (stored by the r-update kernel)
    double alpha_prev, beta_prev;
    double bnorm;       // ||b|| (FP64)
    double tolb;        // tol * ||b||
    int done;           // every shift of this system met its tolerance (or maxiter)
    int iters;          // iterations completed by this system
    int base;           // index of the shift with offset 0
    int blk_steps;      // iterations this system completed in the current block
    // After a residual replacement r is no longer the residual p was built
    // from, so <r, p> != <r, r>: the first step then takes the exact line
    // search alpha = <r, p> / <p, A p> (replaced = 1, alpha_num = <r, p>).
    // Any alpha keeps the three-term residual recurrence, so the shifted
    // systems stay collinear with the base one.
    double alpha_num;
    int replaced;
    // FP64 head of a MIXED solve: the relative threshold until kFinInit, then
    // head_rr = (threshold * ||b||)^2; the head ends once rr <= head_rr.
    double head_rr;
};

// zeta_i(k+1) of a shift with offset `off` from the base step's alpha and
// the previous step's alpha and beta (Sec. 4.3, the shifted-system
// recurrence; alpha_prev = 1, beta_prev = 0 and zeta = zeta_prev = 1 at k = 0).
__host__ __device__ inline double shift_zeta_next(double zeta, double zeta_prev, double alpha,
                                                  double alpha_prev, double beta_prev, double off) {
    return zeta * zeta_prev * alpha_prev /
           (zeta_prev * alpha_prev * (1.0 + alpha * off) + alpha * beta_prev * (zeta_prev - zeta));
}

// Numerator of alpha for step q of the current block.
__host__ __device__ inline double step_alpha_num(const SysScalars& s, int q) {
    return s.replaced ? s.alpha_num : s.rr[q & 1];
}

// Shifted solutions are not touched every iteration.  Inside a block of
// iterations starting at k0 the recurrences of shift i,
//   x_i(k+1) = x_i(k) + a_i(k) p_i(k),   p_i(k+1) = zeta_i(k+1) r(k+1) + b_i(k) p_i(k),
// only record their scalars; at the block boundary they are folded into
// coefficients on P = p_i(k0), X = x_i(k0) and the stored base residuals
// r(k0+1..k0+q):
//   p_i(k0+q) = c P + sum_l d[l] r(k0+l)
//   x_i(k0+q) = X + e P + sum_l f[l] r(k0+l)
struct ShiftScalars {
    double off;                 // sigma_i - sigma_0 >= 0
    double zeta, zeta_prev;
    int active;                 // still iterating
    int block_active;           // active when the current block started
    int conv_iter;
    int nsteps;                 // steps of the current block applied to this shift
};

// Per-step scalars of one shift in the current block (index m = k - k0) and
// the block coefficients computed from them (flush_coefficients).
struct BlockCoef {
    double a[kMaxBlockLen];
    double b[kMaxBlockLen];
    double z[kMaxBlockLen + 1];   // z[l] = zeta_i(k0 + l)
    double c, e;
    double d[kMaxBlockLen + 1];
    double f[kMaxBlockLen + 1];
};

struct SolverState {
    int nsys, nshift;
    int blk_it;        // iterations completed inside the current block
    int all_done;
    int head_done;     // every system done or below its head_rr (read with all_done)
    int first_block;   // P = r(k0) and X = 0 (nothing stored yet)
    int iter;          // iterations completed by the shared solve
    int maxiter;
    int reliable_count;
    BlockCoef* coef;   // device [kMaxSys][kMaxShift]
    // When set, every step of system j records (alpha, beta, <r', r'>) at
    // hist[(j * hist_cap + k) * 3] (k < hist_cap): the scalars the two-pass
    // rational apply rebuilds its weights from.
    double* hist;
    int hist_cap;
    // largest rr / tolb^2 over the systems still iterating (0 once all are
    // done): the host extrapolates it to stop launching blocks once the one
    // in flight should finish the solve
    double conv_ratio;
    SysScalars sys[kMaxSys];
    ShiftScalars sh[kMaxSys][kMaxShift];
};

enum FinalizeKind {
    kFinNone = 0,
    kFinInit = 1,      // after the start kernel: ||b||, rr
    kFinReliable = 4,  // after r = b - A x in FP64: rr
    kFinNorms = 5,     // plain per-rhs sums into an output array
    kFinReliableDot = 6  // after the replacement: <r, p>, the next step's alpha numerator
};

#if defined(__HIPCC__)

// Sum partial[r*nblk + 0..nblk-1] over all threads of the block, in a fixed
// order (so every block that calls it gets the same bits).
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

// Sum rows 0..nrows-1 of partial[r*nblk + b] over b for all rows in one pass
// (fixed order: the same bits in every block that calls it); out[r] in shared
// memory holds the sums on return.  nrows <= MAXR <= kMaxSys.  A thread adds
// its entries b = tid, tid + blockDim, ... in that order; the loads of U of
// them are issued together before they are added, so one memory round trip
// serves U entries (the update kernels sum thousands of operator-block
// partials per system; the many-row form keeps U = 1 for its registers).
template <int MAXR = kMaxSys, int U = (MAXR <= 2 ? 8 : 1)>
__device__ inline void block_sum_rows(const double* partial, int nrows, int nblk, double* out) {
    __shared__ double wsum[MAXR][16];
    double acc[MAXR];
#pragma unroll
    for (int r = 0; r < MAXR; ++r) acc[r] = 0.0;
    const int bd = (int)blockDim.x;
    for (int b = threadIdx.x; b < nblk; b += U * bd) {
        double v[U][MAXR];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                v[u][r] = (r < nrows && b + u * bd < nblk) ? partial[(size_t)r * nblk + b + u * bd] : 0.0;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int r = 0; r < MAXR; ++r)
                if (r < nrows && b + u * bd < nblk) acc[r] += v[u][r];
    }
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int r = 0; r < MAXR; ++r) {
        if (r < nrows) {
            double v = acc[r];
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
            if (lane == 0) wsum[r][wid] = v;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < nrows) {
        const int nw = blockDim.x >> 6;
        double t = 0.0;
        for (int w = 0; w < nw; ++w) t += wsum[threadIdx.x][w];
        out[threadIdx.x] = t;
    }
    __syncthreads();
}

// One-block finalize for the rare reductions (start, reliable update, norms).
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
            s.rr[0] = s.rr[1] = sums[nsys + tid];
            s.head_rr = s.head_rr * s.head_rr * b2;
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
    if (kind == kFinReliableDot) {
        if (tid < nsys && !st->sys[tid].done) {
            st->sys[tid].alpha_num = sums[tid];
            st->sys[tid].replaced = 1;
        }
        return;
    }
    // kFinReliable: the residual was replaced at a block boundary (slot 0)
    if (tid < nsys && !st->sys[tid].done) st->sys[tid].rr[0] = sums[tid];
    if (tid == 0) st->reliable_count += 1;
}

// The FP64 recurrences of one CG step q of the current block (a block of the
// p-update kernel with no vector work runs this while the others update p):
//   alpha = rr / <p, A p>, zeta_i', alpha_i, beta = rr' / rr, beta_i,
//   the step's scalars of every shift, convergence and counters.
// rr for step q is in rr[q & 1]; the new one goes to rr[(q + 1) & 1], which no
// kernel of this step reads.
__device__ inline void iteration_update(SolverState* st, const double* partR, int nblkR,
                                        int q_step) {
    __shared__ double pap_s[kMaxSys], rrn_s[kMaxSys];
    __shared__ int alive_s[kMaxSys];
    const int nsys = st->nsys, nsh = st->nshift;
    const int cur = q_step & 1, nxt = cur ^ 1;
    block_sum_rows(partR, nsys, nblkR, rrn_s);
    if ((int)threadIdx.x < nsys) {
        pap_s[threadIdx.x] = st->sys[threadIdx.x].pap;
        alive_s[threadIdx.x] = 0;
    }
    __syncthreads();
    const int tid = threadIdx.x;
    for (int p = tid; p < nsys * nsh; p += blockDim.x) {
        const int j = p / nsh, i = p % nsh;
        const SysScalars& s = st->sys[j];
        ShiftScalars& h = st->sh[j][i];
        if (s.done || !h.active) continue;
        const double rr = s.rr[cur];
        const double alpha = step_alpha_num(s, q_step) / pap_s[j];
        const double beta = rrn_s[j] / rr;
        const double zeta = h.zeta, zeta_prev = h.zeta_prev;
        const double zn = shift_zeta_next(zeta, zeta_prev, alpha, s.alpha_prev, s.beta_prev, h.off);
        const double ratio = zn / zeta;
        const int q = s.blk_steps;   // this step's index inside the block (0-based)
        BlockCoef& bc = st->coef[j * kMaxShift + i];
        bc.a[q] = alpha * ratio;
        bc.b[q] = beta * ratio * ratio;
        bc.z[q + 1] = zn;
        h.nsteps = q + 1;
        h.zeta_prev = zeta;
        h.zeta = zn;
        if (fabs(zn) * sqrt(rrn_s[j]) <= s.tolb) {
            h.active = 0;
            h.conv_iter = s.iters + 1;
        }
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
            const double rr = s.rr[cur];
            s.alpha_prev = step_alpha_num(s, q_step) / pap_s[tid];
            s.beta_prev = rrn_s[tid] / rr;
            if (st->hist && s.iters < st->hist_cap) {
                double* hp = st->hist + ((size_t)tid * st->hist_cap + s.iters) * 3;
                hp[0] = s.alpha_prev;
                hp[1] = s.beta_prev;
                hp[2] = rrn_s[tid];
            }
            s.replaced = 0;
            s.rr[nxt] = rrn_s[tid];
            s.iters += 1;
            s.blk_steps += 1;
            if (!alive_s[tid] || s.iters >= st->maxiter || !isfinite(rrn_s[tid])) s.done = 1;
        }
    }
    __syncthreads();
    if (tid == 0) {
        int all = 1, head = 1;
        double ratio = 0.0;
        for (int j = 0; j < nsys; ++j) {
            const SysScalars& s = st->sys[j];
            all &= s.done;
            head &= s.done || s.rr[nxt] <= s.head_rr;
            if (!s.done && s.tolb > 0.0) ratio = fmax(ratio, s.rr[nxt] / (s.tolb * s.tolb));
        }
        st->all_done = all;
        st->head_done = head;
        st->conv_ratio = ratio;
        st->blk_it += 1;
        st->iter += 1;
    }
}

// Block coefficients of one shift from its recorded steps m = 0..q-1
// (backward recursions, all terms positive; d[l] = f[l] = 0 for l > q):
//   B_q = 1, B_m = b[m] B_{m+1};   G_q = 0, G_m = a[m] + b[m] G_{m+1}
//   c = B_0, e = G_0, d[l] = z[l] B_l, f[l] = z[l] G_l.
__device__ inline void flush_coefficients(BlockCoef& bc, int q) {
    for (int l = q + 1; l <= kMaxBlockLen; ++l) bc.d[l] = bc.f[l] = 0.0;
    double B = 1.0, G = 0.0;
    for (int m = q - 1; m >= 0; --m) {
        bc.d[m + 1] = bc.z[m + 1] * B;
        bc.f[m + 1] = bc.z[m + 1] * G;
        G = bc.a[m] + bc.b[m] * G;
        B = bc.b[m] * B;
    }
    bc.c = B;
    bc.e = G;
}

#endif  // __HIPCC__

}  // namespace rhmc
