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
    const int j = blockIdx.y;
    double r2 = 0.0;
    const bool live = !st->sys[j].done;
    const double alpha = st->sys[j].alpha;
    for (size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2; live && i < a.n;
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
    reduce_store(r2, 0.0, j, -1, a.partial);
}

// ------------------------------------------------------------------ p update
// p(k+1) = r(k+1) + beta p(k)
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_pupdate(VecArgs<VT> a) {
    const SolverState* st = reinterpret_cast<const SolverState*>(a.state);
    if (st->all_done) return;
    const int j = blockIdx.y;
    if (st->sys[j].done) return;
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2;
    if (i >= a.n) return;
    const double beta = st->sys[j].beta_prev;
    Pair<VT> r, p;
    r.load(a.x[j], i);
    p.load(a.y[j], i);
    for (int k = 0; k < 2; ++k) {
        p.re[k] = (double)r.re[k] + beta * (double)p.re[k];
        p.im[k] = (double)r.im[k] + beta * (double)p.im[k];
    }
    p.store(a.y[j], i);
}

// ------------------------------------------------------------------ flush
// Apply the coefficients accumulated since the last block boundary:
//   X_i <- X_i + e P_i + sum_l f[l] r_l,   P_i <- c P_i + sum_l d[l] r_l
// for every shift active when the block started, then r_0 <- r_q and reset.
template <typename VT, int Q>
__device__ __forceinline__ void flush_site(const FlushArgs<VT>& a, const SolverState* st, int j,
                                           size_t i) {
    const SysScalars& s = st->sys[j];
    const int q = s.blk_steps;
    Pair<VT> rl[Q + 1];
#pragma unroll
    for (int l = 0; l <= Q; ++l)
        if (l <= q) rl[l].load(a.ring[l][j], i);
    const int first = st->first_block;
    for (int sh = 0; sh < st->nshift; ++sh) {
        const ShiftScalars& h = st->sh[j][sh];
        if (!h.block_active) continue;
        Pair<VT> P;
        Pair<double2> X;
        if (first) {
            P = rl[0];
            X.re[0] = X.re[1] = X.im[0] = X.im[1] = 0.0;
        } else {
            P.load(a.P + ((size_t)j * a.nshift + sh) * a.n, i);
            X.load(a.X + j * a.x_sys + sh * a.x_shift, i);
        }
        double xr[2], xi[2], pr[2], pi[2];
        for (int k = 0; k < 2; ++k) {
            xr[k] = X.re[k] + h.e * (double)P.re[k];
            xi[k] = X.im[k] + h.e * (double)P.im[k];
            pr[k] = h.c * (double)P.re[k];
            pi[k] = h.c * (double)P.im[k];
        }
#pragma unroll
        for (int l = 1; l <= Q; ++l) {
            if (l > q) break;
            const double f = h.f[l], d = h.d[l];
            for (int k = 0; k < 2; ++k) {
                xr[k] += f * (double)rl[l].re[k];
                xi[k] += f * (double)rl[l].im[k];
                pr[k] += d * (double)rl[l].re[k];
                pi[k] += d * (double)rl[l].im[k];
            }
        }
        for (int k = 0; k < 2; ++k) {
            X.re[k] = xr[k];
            X.im[k] = xi[k];
        }
        X.store(a.X + j * a.x_sys + sh * a.x_shift, i);
        if (h.active) {
            for (int k = 0; k < 2; ++k) {
                P.re[k] = pr[k];
                P.im[k] = pi[k];
            }
            P.store(a.P + ((size_t)j * a.nshift + sh) * a.n, i);
        }
    }
    if (q > 0) rl[q > Q ? Q : q].store(a.ring[0][j], i);
}

template <typename VT, int Q>
__global__ __launch_bounds__(kBlock) void k_flush(FlushArgs<VT> a) {
    const SolverState* st = reinterpret_cast<const SolverState*>(a.state);
    const int j = blockIdx.y;
    const size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2;
    if (st->sys[j].blk_steps > 0 && i < a.n) flush_site<VT, Q>(a, st, j, i);
}

// After a flush: restart the block coefficients (one block).
__global__ __launch_bounds__(kBlock) void k_flush_reset(void* state) {
    SolverState* st = reinterpret_cast<SolverState*>(state);
    const int nsys = st->nsys, nsh = st->nshift;
    for (int p = threadIdx.x; p < nsys * nsh; p += blockDim.x) {
        ShiftScalars& h = st->sh[p / nsh][p % nsh];
        h.c = 1.0;
        h.e = 0.0;
        for (int l = 0; l <= kMaxBlockLen; ++l) h.d[l] = h.f[l] = 0.0;
        h.block_active = h.active;
    }
    __syncthreads();
    if (threadIdx.x < nsys) st->sys[threadIdx.x].blk_steps = 0;
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
constexpr int kRedBlocks = 1024;
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
    hipLaunchKernelGGL(k_pupdate<VT>, vec_grid(a.n, nsys), dim3(kBlock), 0, s, a);
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
    const dim3 g = vec_grid(a.n, nsys), b(kBlock);
    if (qmax <= 4)
        hipLaunchKernelGGL((k_flush<VT, 4>), g, b, 0, s, a);
    else if (qmax <= 8)
        hipLaunchKernelGGL((k_flush<VT, 8>), g, b, 0, s, a);
    else if (qmax <= 12)
        hipLaunchKernelGGL((k_flush<VT, 12>), g, b, 0, s, a);
    else
        hipLaunchKernelGGL((k_flush<VT, 16>), g, b, 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
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
