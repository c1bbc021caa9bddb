// BLAS-1 kernels of the multi-shift CG (Sec. 4.3) and the rational combine
// (Eq. system_r).  Each kernel streams one or more colour vectors once; the
// ones that feed a CG scalar also emit one partial sum per block and let the
// last block run the FP64 recurrences (state.h).
//
// Vectors of a system are flat arrays of n = 3*Vh complex numbers; a thread
// handles two consecutive complex numbers (one 16-byte load in FP32).
#include "blas.h"
#include "state.h"

namespace rhmc {

template <typename VT> struct Pair;
template <> struct Pair<float2> {
    float re[2], im[2];
    __device__ __forceinline__ void load(const float2* p, size_t i) {
        const float4 v = *reinterpret_cast<const float4*>(p + i);
        re[0] = v.x; im[0] = v.y; re[1] = v.z; im[1] = v.w;
    }
    __device__ __forceinline__ void store(float2* p, size_t i) const {
        *reinterpret_cast<float4*>(p + i) = make_float4(re[0], im[0], re[1], im[1]);
    }
};
template <> struct Pair<double2> {
    double re[2], im[2];
    __device__ __forceinline__ void load(const double2* p, size_t i) {
        const double2 a = p[i], b = p[i + 1];
        re[0] = a.x; im[0] = a.y; re[1] = b.x; im[1] = b.y;
    }
    __device__ __forceinline__ void store(double2* p, size_t i) const {
        p[i] = make_double2(re[0], im[0]);
        p[i + 1] = make_double2(re[1], im[1]);
    }
};

// Block-reduce up to two doubles and store them as partial[r*gridDim.x + bx]
// (r0, r1 >= 0).  The sums are finished by a one-block finalize kernel: the
// kernel boundary makes every partial visible, with no per-block fence.
__device__ __forceinline__ void reduce_store(double v0, double v1, int r0, int r1,
                                             double* partial) {
    __shared__ double sm[2][kBlock / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int off = 32; off > 0; off >>= 1) {
        v0 += __shfl_xor(v0, off, 64);
        v1 += __shfl_xor(v1, off, 64);
    }
    if (lane == 0) {
        sm[0][wid] = v0;
        sm[1][wid] = v1;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        const int r = threadIdx.x == 0 ? r0 : r1;
        if (r >= 0) {
            double s = 0.0;
            for (int w = 0; w < kBlock / 64; ++w) s += sm[threadIdx.x][w];
            partial[(size_t)r * gridDim.x + blockIdx.x] = s;
        }
    }
}

// ------------------------------------------------------------------ finalize
// One block: finish the block sums of the preceding kernel and run the FP64
// scalar recurrences of the multi-shift CG (state.h).
__global__ __launch_bounds__(kBlock) void k_finalize(int kind, void* state, const double* partial,
                                                     int nblk, int nrhs, double* out_sums) {
    if (kind != kFinNorms && kind != kFinInit &&
        reinterpret_cast<const SolverState*>(state)->all_done)
        return;
    solver_finalize(kind, state, partial, nblk, nrhs, out_sums);
}

// ------------------------------------------------------------------ start
// r(0) = p = b (rounded to the iteration precision); sums ||b||^2 and ||r(0)||^2.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_start(VecArgs<VT> a) {
    SolverState* st = reinterpret_cast<SolverState*>(a.state);
    const int j = blockIdx.y;
    double b2 = 0.0, r2 = 0.0;
    for (size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2; i < a.n;
         i += (size_t)gridDim.x * kBlock * 2) {
        Pair<double2> b;
        b.load(a.b64[j], i);
        Pair<VT> r;
        for (int k = 0; k < 2; ++k) {
            r.re[k] = b.re[k];
            r.im[k] = b.im[k];
            b2 += b.re[k] * b.re[k] + b.im[k] * b.im[k];
            r2 += (double)r.re[k] * r.re[k] + (double)r.im[k] * r.im[k];
        }
        r.store(a.x[j], i);
        r.store(a.y[j], i);
    }
    reduce_store(b2, r2, j, st->nsys + j, a.partial);
}

// ------------------------------------------------------------------ r update
// r(k+1) = r(k) - alpha A p;  sum ||r(k+1)||^2  -> beta, shift recurrences.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_rupdate(VecArgs<VT> a) {
    SolverState* st = reinterpret_cast<SolverState*>(a.state);
    if (st->all_done) return;
    __shared__ double smem[16];
    const int j = blockIdx.y;
    const bool live = !st->sys[j].done;
    double r2 = 0.0;
    if (live) {
        // alpha = rr / <p, A p>; every block adds the A-kernel partials itself,
        // in the same fixed order, so all blocks use the same alpha bits
        const double pap = block_sum_partials(a.part2, j, a.nblk2, smem);
        const double alpha = st->sys[j].rr[a.q & 1] / pap;
        for (size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2; i < a.n;
             i += (size_t)gridDim.x * kBlock * 2) {
            Pair<VT> r, ap;
            r.load(a.x[j], i);
            ap.load(a.y[j], i);
            for (int k = 0; k < 2; ++k) {
                const double nr = (double)r.re[k] - alpha * (double)ap.re[k];
                const double ni = (double)r.im[k] - alpha * (double)ap.im[k];
                r.re[k] = nr;
                r.im[k] = ni;
                r2 += (double)r.re[k] * r.re[k] + (double)r.im[k] * r.im[k];
            }
            r.store(a.z[j], i);
        }
    }
    reduce_store(r2, 0.0, j, -1, a.partial);
}

// ------------------------------------------------------------------ p update
// p(k+1) = r(k+1) + beta p(k); block (0, 0) also runs the FP64 recurrences
// of this step (iteration_update), which the other blocks do not read.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_pupdate(VecArgs<VT> a) {
    SolverState* st = reinterpret_cast<SolverState*>(a.state);
    __shared__ double smem[16];
    __shared__ int flags[2];
    const int j = blockIdx.y;
    // Block (0, 0) writes done / all_done during this kernel: every other block
    // reads them once, through shared memory, so its threads agree on the
    // branches around the barriers below.
    if (threadIdx.x == 0) {
        flags[0] = st->all_done;
        flags[1] = st->sys[j].done;
    }
    __syncthreads();
    if (flags[0]) return;
    if (!flags[1]) {
        const double rrn = block_sum_partials(a.partial, j, a.nblk, smem);
        const double beta = rrn / st->sys[j].rr[a.q & 1];
        for (size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2; i < a.n;
             i += (size_t)gridDim.x * kBlock * 2) {
            Pair<VT> r, p;
            r.load(a.x[j], i);
            p.load(a.y[j], i);
            for (int k = 0; k < 2; ++k) {
                p.re[k] = (double)r.re[k] + beta * (double)p.re[k];
                p.im[k] = (double)r.im[k] + beta * (double)p.im[k];
            }
            p.store(a.y[j], i);
        }
    }
    if (blockIdx.x == 0 && blockIdx.y == 0) {
        __syncthreads();
        iteration_update(st, a.part2, a.nblk2, a.partial, a.nblk, a.q);
    }
}

// ------------------------------------------------------------------ flush
// Block coefficients of every shift that took part in the block (one block,
// one thread per (system, shift)); run before k_flush.
__global__ __launch_bounds__(kBlock) void k_flush_coef(void* state) {
    SolverState* st = reinterpret_cast<SolverState*>(state);
    const int nsys = st->nsys, nsh = st->nshift;
    for (int p = threadIdx.x; p < nsys * nsh; p += blockDim.x) {
        const int j = p / nsh, i = p % nsh;
        const ShiftScalars& h = st->sh[j][i];
        if (h.block_active) flush_coefficients(st->coef[j * kMaxShift + i], h.nsteps);
    }
}

template <typename VT> struct Comp;
template <> struct Comp<float2> { using type = float; };
template <> struct Comp<double2> { using type = double; };

// One thread per complex element of one system's vectors: the q+1 stored base
// residuals stay in registers while every shift's X and P stream through
// once.  Shifts go in chunks of U: their loads are issued together, then each
// residual is widened to FP64 once and applied to all U shifts.
template <typename VT, int Q>
__global__ __launch_bounds__(kBlock) void k_flush(FlushArgs<VT> a) {
    using RT = typename Comp<VT>::type;
    constexpr int U = (sizeof(VT) == 16 && Q > 16) ? 2 : 4;
    const SolverState* st = reinterpret_cast<const SolverState*>(a.state);
    const BlockCoef* coef = reinterpret_cast<const BlockCoef*>(a.coef);
    const int j = blockIdx.y;
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    const int q = st->sys[j].blk_steps;
    if (q == 0 || i >= a.n) return;
    RT rre[Q + 1], rim[Q + 1];
#pragma unroll
    for (int l = 0; l <= Q; ++l)
        if (l <= q) {
            const VT v = a.ring[((size_t)l * a.nsys + j) * a.n + i];
            rre[l] = v.x;
            rim[l] = v.y;
        }
    const bool first = st->first_block != 0;
    const int nsh = a.nshift;
    for (int s0 = 0; s0 < nsh; s0 += U) {
        // keep the widening of the residuals inside this chunk (not hoisted
        // out of the shift loop, which would hold them all as FP64)
#pragma unroll
        for (int l = 0; l <= Q; ++l) asm volatile("" : "+v"(rre[l]), "+v"(rim[l]));
        bool act[U];
        int qi[U];
        double xr[U], xi[U], pr[U], pi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int sh = s0 + u;
            act[u] = sh < nsh && st->sh[j][sh].block_active;
            qi[u] = act[u] ? st->sh[j][sh].nsteps : 0;
            xr[u] = xi[u] = pr[u] = pi[u] = 0.0;
            if (act[u]) {
                double p0r, p0i;
                if (first) {
                    p0r = (double)rre[0];
                    p0i = (double)rim[0];
                } else {
                    const double2 x = a.X[j * a.x_sys + sh * a.x_shift + i];
                    const VT p = a.P[((size_t)j * nsh + sh) * a.n + i];
                    xr[u] = x.x;
                    xi[u] = x.y;
                    p0r = (double)p.x;
                    p0i = (double)p.y;
                }
                const BlockCoef& bc = coef[j * kMaxShift + sh];
                xr[u] += bc.e * p0r;
                xi[u] += bc.e * p0i;
                pr[u] = bc.c * p0r;
                pi[u] = bc.c * p0i;
            }
        }
#pragma unroll
        for (int l = 1; l <= Q; ++l) {
            if (l <= q) {
                const double rr = (double)rre[l], ri = (double)rim[l];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    if (l <= qi[u]) {
                        const BlockCoef& bc = coef[j * kMaxShift + s0 + u];
                        const double f = bc.f[l], d = bc.d[l];
                        xr[u] += f * rr;
                        xi[u] += f * ri;
                        pr[u] += d * rr;
                        pi[u] += d * ri;
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!act[u]) continue;
            const int sh = s0 + u;
            a.X[j * a.x_sys + sh * a.x_shift + i] = make_double2(xr[u], xi[u]);
            if (st->sh[j][sh].active) {
                VT pv;
                pv.x = (RT)pr[u];
                pv.y = (RT)pi[u];
                a.P[((size_t)j * nsh + sh) * a.n + i] = pv;
            }
        }
    }
    // the last stored residual is r(k0) of the next block
#pragma unroll
    for (int l = 1; l <= Q; ++l)
        if (l == q) {
            VT v;
            v.x = rre[l];
            v.y = rim[l];
            a.ring[(size_t)j * a.n + i] = v;
        }
}

// After a flush: restart the block bookkeeping (one block).
__global__ __launch_bounds__(kBlock) void k_flush_reset(void* state) {
    SolverState* st = reinterpret_cast<SolverState*>(state);
    const int nsys = st->nsys, nsh = st->nshift;
    for (int p = threadIdx.x; p < nsys * nsh; p += blockDim.x) {
        ShiftScalars& h = st->sh[p / nsh][p % nsh];
        h.nsteps = 0;
        h.block_active = h.active;
    }
    __syncthreads();
    if (threadIdx.x < nsys) {
        SysScalars& s = st->sys[threadIdx.x];
        if (st->blk_it & 1) s.rr[0] = s.rr[1];   // the next block starts at step 0
        s.blk_steps = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st->first_block = 0;
        st->blk_it = 0;
    }
}

// ------------------------------------------------------------------ combine
// y = alpha0 b + sum_i alpha_i x_i  (FP64)
__global__ __launch_bounds__(kBlock) void k_combine(CombineArgs a) {
    const int j = blockIdx.y;
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2;
    if (i >= a.n) return;
    Pair<double2> b, y;
    b.load(a.b[j], i);
    for (int k = 0; k < 2; ++k) {
        y.re[k] = a.alpha0 * b.re[k];
        y.im[k] = a.alpha0 * b.im[k];
    }
    for (int s = 0; s < a.nterm; ++s) {
        Pair<double2> x;
        x.load(a.x[j] + (size_t)s * a.x_stride, i);
        for (int k = 0; k < 2; ++k) {
            y.re[k] += a.alpha[s] * x.re[k];
            y.im[k] += a.alpha[s] * x.im[k];
        }
    }
    y.store(a.y[j], i);
}

// ------------------------------------------------------------------ axpy
// y += x (FP64), for folding a correction into a solution
__global__ __launch_bounds__(kBlock) void k_add(AddArgs a) {
    const int j = blockIdx.y;
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2;
    if (i >= a.n) return;
    Pair<double2> x, y;
    x.load(a.x[j], i);
    y.load(a.y[j], i);
    for (int k = 0; k < 2; ++k) {
        y.re[k] += x.re[k];
        y.im[k] += x.im[k];
    }
    y.store(a.y[j], i);
}

// ------------------------------------------------------------------ launchers
static dim3 vec_grid(size_t n, int nsys) {
    return dim3((unsigned)((n / 2 + kBlock - 1) / kBlock), (unsigned)nsys);
}

// reducing kernels stride over the vector with at most kRedBlocks blocks per
// system, which bounds the number of partial sums the finalize has to add
constexpr int kRedBlocks = 512;
static dim3 red_grid(size_t n, int nsys) { return dim3((unsigned)vec_blocks(n), (unsigned)nsys); }

template <typename VT>
hipError_t launch_start(const VecArgs<VT>& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_start<VT>, red_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
template <typename VT>
hipError_t launch_rupdate(const VecArgs<VT>& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_rupdate<VT>, red_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
template <typename VT>
hipError_t launch_pupdate(const VecArgs<VT>& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_pupdate<VT>, red_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
int vec_blocks(size_t n) {
    const size_t full = (n / 2 + kBlock - 1) / kBlock;
    return (int)(full < (size_t)kRedBlocks ? full : (size_t)kRedBlocks);
}

hipError_t launch_finalize(int kind, void* state, const double* partial, int nblk, int nrhs,
                           double* out_sums, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(kBlock), 0, s, kind, state, partial, nblk, nrhs,
                       out_sums);
    return hipGetLastError();
}

template <typename VT>
hipError_t launch_flush(const FlushArgs<VT>& a, int nsys, int qmax, hipStream_t s) {
    hipLaunchKernelGGL(k_flush_coef, dim3(1), dim3(kBlock), 0, s, a.state);
    const dim3 g((unsigned)((a.n + kBlock - 1) / kBlock), (unsigned)nsys), b(kBlock);
    if (qmax <= 4)
        hipLaunchKernelGGL((k_flush<VT, 4>), g, b, 0, s, a);
    else if (qmax <= 8)
        hipLaunchKernelGGL((k_flush<VT, 8>), g, b, 0, s, a);
    else if (qmax <= 16)
        hipLaunchKernelGGL((k_flush<VT, 16>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((k_flush<VT, 32>), g, b, 0, s, a);
    hipLaunchKernelGGL(k_flush_reset, dim3(1), dim3(kBlock), 0, s, a.state);
    return hipGetLastError();
}
hipError_t launch_combine(const CombineArgs& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, vec_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_add(const AddArgs& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_add, vec_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template hipError_t launch_start<float2>(const VecArgs<float2>&, int, hipStream_t);
template hipError_t launch_start<double2>(const VecArgs<double2>&, int, hipStream_t);
template hipError_t launch_rupdate<float2>(const VecArgs<float2>&, int, hipStream_t);
template hipError_t launch_rupdate<double2>(const VecArgs<double2>&, int, hipStream_t);
template hipError_t launch_pupdate<float2>(const VecArgs<float2>&, int, hipStream_t);
template hipError_t launch_pupdate<double2>(const VecArgs<double2>&, int, hipStream_t);
template hipError_t launch_flush<float2>(const FlushArgs<float2>&, int, int, hipStream_t);
template hipError_t launch_flush<double2>(const FlushArgs<double2>&, int, int, hipStream_t);

}  // namespace rhmc
