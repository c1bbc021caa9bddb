// BLAS-1 kernels of the multi-shift CG (Sec. 4.3) and the rational combine
// (Eq. system_r).  Each kernel streams one or more colour vectors once; the
// ones that feed a CG scalar also emit one partial sum per block, which the
// blocks of the next kernel add up themselves (block 0 of the p-update runs
// the FP64 recurrences, state.h).
//
// Vectors of a system are flat arrays of n = 3*Vh complex numbers; a thread
// handles two consecutive complex numbers (one 16-byte load in FP32).
#include <type_traits>

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

// Entries i and i + 1 of one system of an FP32 set whose systems are paired
// (every other complex64, f32_offset); FP64 sets are never paired.
template <typename VT>
__device__ __forceinline__ void load_sys(Pair<VT>& u, const VT* p, size_t i, int paired) {
    if (!paired) {
        u.load(p, i);
        return;
    }
    const VT a = p[i << 1], b = p[(i + 1) << 1];
    u.re[0] = a.x; u.im[0] = a.y; u.re[1] = b.x; u.im[1] = b.y;
}
template <typename VT>
__device__ __forceinline__ void store_sys(const Pair<VT>& v, VT* p, size_t i, int paired) {
    if (!paired) {
        v.store(p, i);
        return;
    }
    VT a, b;
    a.x = v.re[0]; a.y = v.im[0]; b.x = v.re[1]; b.y = v.im[1];
    p[i << 1] = a;
    p[(i + 1) << 1] = b;
}

// Block-reduce up to two doubles and store them as partial[r*gridDim.x + bx]
// (r0, r1 >= 0).  The sums are finished in a later kernel (the next update's
// blocks or a one-block finalize): the kernel boundary makes every partial
// visible, with no per-block fence.
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
        store_sys(r, a.x[j], i, a.paired);
        store_sys(r, a.y[j], i, a.paired);
    }
    reduce_store(b2, r2, j, st->nsys + j, a.partial);
}

// ------------------------------------------------------------------ r update
// Vector kernels stride over the pairs of a system with kUnroll pairs per
// thread per pass, all loads of a pass issued before its stores.
constexpr int kUnroll = 4;

// r(k+1) = r(k) - alpha A p;  sum ||r(k+1)||^2  -> beta, shift recurrences.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_rupdate(VecArgs<VT> a) {
    SolverState* st = reinterpret_cast<SolverState*>(a.state);
    if (st->all_done) return;
    __shared__ double sums[kMaxSys];
    const int j = blockIdx.y;
    const bool live = !st->sys[j].done;
    double r2 = 0.0;
    if (live) {
        const VT* __restrict__ x = a.x[j];
        const VT* __restrict__ y = a.y[j];
        VT* __restrict__ z = a.z[j];
        const size_t stride = (size_t)gridDim.x * kBlock * 2;
        size_t i0 = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2;
        Pair<VT> r[kUnroll], ap[kUnroll];
        auto load_pass = [&]() {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const size_t i = i0 + u * stride;
                if (i < a.n) {
                    r[u].load(x, i);
                    ap[u].load(y, i);
                }
            }
        };
        // the first pass's loads do not depend on alpha: they go out before
        // the block sums, so the two memory round trips overlap
        load_pass();
        // alpha = rr / <p, A p> (<r, p> / <p, A p> right after a residual
        // replacement); every block adds the A-kernel partials itself, in the
        // same fixed order, so all blocks use the same alpha bits
        block_sum_rows<1>(a.part2 + (size_t)j * a.nblk2, 1, a.nblk2, sums);
        const double pap = sums[0];
        if (blockIdx.x == 0 && threadIdx.x == 0) st->sys[j].pap = pap;
        const double alpha = step_alpha_num(st->sys[j], a.q) / pap;
        for (bool first = true; i0 < a.n; i0 += stride * kUnroll, first = false) {
            if (!first) load_pass();
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const size_t i = i0 + u * stride;
                if (i < a.n) {
                    for (int k = 0; k < 2; ++k) {
                        const double nr = (double)r[u].re[k] - alpha * (double)ap[u].re[k];
                        const double ni = (double)r[u].im[k] - alpha * (double)ap[u].im[k];
                        r[u].re[k] = nr;
                        r[u].im[k] = ni;
                        r2 += (double)r[u].re[k] * r[u].re[k] + (double)r[u].im[k] * r[u].im[k];
                    }
                    r[u].store(z, i);
                }
            }
        }
    }
    reduce_store(r2, 0.0, j, -1, a.partial);
}

// ------------------------------------------------------------------ p update
// p(k+1) = r(k+1) + beta p(k).  Block x = 0 of system 0 has no vector work:
// it runs the FP64 recurrences of this step (iteration_update), which no
// other block of this kernel reads; blocks x = 0 of the other systems idle.
template <typename VT>
__global__ __launch_bounds__(kBlock) void k_pupdate(VecArgs<VT> a) {
    SolverState* st = reinterpret_cast<SolverState*>(a.state);
    __shared__ double sums[kMaxSys];
    __shared__ int flags[2];
    const int j = blockIdx.y;
    // The recurrence block writes done / all_done during this kernel: every
    // other block reads them once, through shared memory, so its threads
    // agree on the branches around the barriers below.
    if (threadIdx.x == 0) {
        flags[0] = st->all_done;
        flags[1] = st->sys[j].done;
    }
    __syncthreads();
    if (flags[0]) return;
    if (blockIdx.x == 0) {
        if (j == 0) iteration_update(st, a.partial, a.nblk, a.q);
        return;
    }
    if (flags[1]) return;
    const VT* __restrict__ x = a.x[j];
    VT* __restrict__ y = a.y[j];
    const size_t stride = (size_t)(gridDim.x - 1) * kBlock * 2;
    size_t i0 = ((size_t)(blockIdx.x - 1) * kBlock + threadIdx.x) * 2;
    Pair<VT> r[kUnroll], p[kUnroll];
    auto load_pass = [&]() {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const size_t i = i0 + u * stride;
            if (i < a.n) {
                r[u].load(x, i);
                p[u].load(y, i);
            }
        }
    };
    load_pass();   // independent of beta: overlaps the block sums
    block_sum_rows<1>(a.partial + (size_t)j * a.nblk, 1, a.nblk, sums);
    const double beta = sums[0] / st->sys[j].rr[a.q & 1];
    for (bool first = true; i0 < a.n; i0 += stride * kUnroll, first = false) {
        if (!first) load_pass();
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const size_t i = i0 + u * stride;
            if (i < a.n) {
                for (int k = 0; k < 2; ++k) {
                    p[u].re[k] = (double)r[u].re[k] + beta * (double)p[u].re[k];
                    p[u].im[k] = (double)r[u].im[k] + beta * (double)p[u].im[k];
                }
                p[u].store(y, i);
            }
        }
    }
}

// ------------------------------------------------------------------ paired FP32 updates
// The same two updates on paired FP32 sets (f32_offset): block row y takes
// systems 2y and 2y + 1, a thread one float4 (one complex entry of both) per
// element; the arithmetic of each entry is that of k_rupdate / k_pupdate.
// The half of a finished system (or the absent partner of an odd count) is
// stored back unchanged.
__global__ __launch_bounds__(kBlock) void k_rupdate_pair(VecArgs<float2> a) {
    SolverState* st = reinterpret_cast<SolverState*>(a.state);
    if (st->all_done) return;
    __shared__ double sums[kMaxSys];
    const int j0 = 2 * (int)blockIdx.y, j1 = j0 + 1;
    const bool has1 = j1 < st->nsys;
    const bool live0 = !st->sys[j0].done, live1 = has1 && !st->sys[j1].done;
    double r2a = 0.0, r2b = 0.0;
    if (live0 || live1) {
        const float4* __restrict__ x = reinterpret_cast<const float4*>(a.x[j0]);
        const float4* __restrict__ y = reinterpret_cast<const float4*>(a.y[j0]);
        float4* __restrict__ z = reinterpret_cast<float4*>(a.z[j0]);
        const size_t stride = (size_t)gridDim.x * kBlock;
        size_t i0 = (size_t)blockIdx.x * kBlock + threadIdx.x;
        float4 r[kUnroll], ap[kUnroll];
        auto load_pass = [&]() {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const size_t i = i0 + u * stride;
                if (i < a.n) {
                    r[u] = x[i];
                    ap[u] = y[i];
                }
            }
        };
        load_pass();   // independent of alpha: overlaps the block sums
        block_sum_rows<2>(a.part2 + (size_t)j0 * a.nblk2, has1 ? 2 : 1, a.nblk2, sums);
        const double pap0 = sums[0], pap1 = has1 ? sums[1] : 1.0;
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            if (live0) st->sys[j0].pap = pap0;
            if (live1) st->sys[j1].pap = pap1;
        }
        const double al0 = live0 ? step_alpha_num(st->sys[j0], a.q) / pap0 : 0.0;
        const double al1 = live1 ? step_alpha_num(st->sys[j1], a.q) / pap1 : 0.0;
        for (bool first = true; i0 < a.n; i0 += stride * kUnroll, first = false) {
            if (!first) load_pass();
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const size_t i = i0 + u * stride;
                if (i < a.n) {
                    if (live0) {
                        r[u].x = (float)((double)r[u].x - al0 * (double)ap[u].x);
                        r[u].y = (float)((double)r[u].y - al0 * (double)ap[u].y);
                        r2a += (double)r[u].x * r[u].x + (double)r[u].y * r[u].y;
                    }
                    if (live1) {
                        r[u].z = (float)((double)r[u].z - al1 * (double)ap[u].z);
                        r[u].w = (float)((double)r[u].w - al1 * (double)ap[u].w);
                        r2b += (double)r[u].z * r[u].z + (double)r[u].w * r[u].w;
                    }
                    z[i] = r[u];
                }
            }
        }
    }
    reduce_store(r2a, r2b, j0, has1 ? j1 : -1, a.partial);
}

__global__ __launch_bounds__(kBlock) void k_pupdate_pair(VecArgs<float2> a) {
    SolverState* st = reinterpret_cast<SolverState*>(a.state);
    __shared__ double sums[kMaxSys];
    __shared__ int flags[3];
    const int j0 = 2 * (int)blockIdx.y, j1 = j0 + 1;
    const bool has1 = j1 < st->nsys;
    // done flags change during this kernel (the recurrence block): read once
    if (threadIdx.x == 0) {
        flags[0] = st->all_done;
        flags[1] = st->sys[j0].done;
        flags[2] = has1 ? st->sys[j1].done : 1;
    }
    __syncthreads();
    if (flags[0]) return;
    if (blockIdx.x == 0) {
        if (blockIdx.y == 0) iteration_update(st, a.partial, a.nblk, a.q);
        return;
    }
    const bool live0 = !flags[1], live1 = !flags[2];
    if (!live0 && !live1) return;
    const float4* __restrict__ x = reinterpret_cast<const float4*>(a.x[j0]);
    float4* __restrict__ y = reinterpret_cast<float4*>(a.y[j0]);
    const size_t stride = (size_t)(gridDim.x - 1) * kBlock;
    size_t i0 = (size_t)(blockIdx.x - 1) * kBlock + threadIdx.x;
    float4 r[kUnroll], p[kUnroll];
    auto load_pass = [&]() {
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const size_t i = i0 + u * stride;
            if (i < a.n) {
                r[u] = x[i];
                p[u] = y[i];
            }
        }
    };
    load_pass();   // independent of beta: overlaps the block sums
    block_sum_rows<2>(a.partial + (size_t)j0 * a.nblk, has1 ? 2 : 1, a.nblk, sums);
    const double beta0 = live0 ? sums[0] / st->sys[j0].rr[a.q & 1] : 0.0;
    const double beta1 = live1 ? sums[1] / st->sys[j1].rr[a.q & 1] : 0.0;
    for (bool first = true; i0 < a.n; i0 += stride * kUnroll, first = false) {
        if (!first) load_pass();
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const size_t i = i0 + u * stride;
            if (i < a.n) {
                if (live0) {
                    p[u].x = (float)((double)r[u].x + beta0 * (double)p[u].x);
                    p[u].y = (float)((double)r[u].y + beta0 * (double)p[u].y);
                }
                if (live1) {
                    p[u].z = (float)((double)r[u].z + beta1 * (double)p[u].z);
                    p[u].w = (float)((double)r[u].w + beta1 * (double)p[u].w);
                }
                y[i] = p[u];
            }
        }
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

// One thread per complex element of one system's vectors: the stored base
// residuals r(k0+l), l <= q, stay in registers while every shift's X and P
// stream through once, a pair of shifts per pass.  The coefficients of a pass
// (e, c, f_l, d_l of both shifts, for each system of the block) are staged in
// LDS and read by broadcast: in scalar registers they would not fit.  The
// coefficients are zero beyond a shift's last step (k_flush_coef), so the
// step loop is straight-line code over l = 1..Q; ring slots beyond q are read
// as slot q (finite values times zero).  Paired FP32 rings: block row y takes
// systems 2y and 2y + 1, the two halves of a block the same elements of both,
// so each 16-byte ring entry is fetched from memory once.
template <typename VT, int Q>
__global__ __launch_bounds__(kBlock) void k_flush(FlushArgs<VT> a,
                                                  const BlockCoef* __restrict__ coef) {
    constexpr int U = 2;
    constexpr int H = kBlock / 2;
    __shared__ double2 cs[2][U][Q + 1];   // [system of the block][u][l]: (f_l, d_l); l = 0: (e, c)
    const SolverState* st = reinterpret_cast<const SolverState*>(a.state);
    const int nsb = a.paired ? 2 : 1;    // systems per block
    int hs = 0;                          // this thread's system within the block
    size_t i;
    if (a.paired) {
        hs = (int)threadIdx.x >= H;
        i = (size_t)blockIdx.x * H + (threadIdx.x - hs * H);
    } else {
        i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    }
    // uniform over a wave (half a block is two whole waves): scalar registers
    hs = __builtin_amdgcn_readfirstlane(hs);
    auto sys_of = [&](int h) { return a.paired ? 2 * (int)blockIdx.y + h : (int)blockIdx.y; };
    auto steps_of = [&](int h) { return sys_of(h) < a.nsys ? st->sys[sys_of(h)].blk_steps : 0; };
    const int j = sys_of(hs);
    const int q = steps_of(hs);
    if (steps_of(0) == 0 && (nsb == 1 || steps_of(1) == 0)) return;   // the whole block
    const bool live = q != 0 && i < a.n;
    // Long blocks keep an FP32 ring in FP32 registers, widened where it is
    // used (below); for 16 to 25 steps that form makes the compiler spill, so
    // shorter rings are widened on load instead.
    using RR = typename std::conditional<std::is_same<VT, float2>::value && (Q >= 32), float,
                                         double>::type;
    RR rre[Q + 1], rim[Q + 1];
    const size_t off = live ? f32_offset(a.paired, j, i, a.n) : 0;
#pragma unroll
    for (int l = 0; l <= Q; ++l) {
        rre[l] = rim[l] = 0.0;
        if (live) {
            const VT v = a.ring[(size_t)(l < q ? l : q) * a.ring_slot + off];
            rre[l] = v.x;
            rim[l] = v.y;
        }
    }
    const bool first = st->first_block != 0;
    const int nsh = a.nshift;
    double2* __restrict__ X = a.X;
    double2* __restrict__ P = a.P;
#pragma unroll 1
    for (int s0 = 0; s0 < nsh; s0 += U) {
        // skip (block-uniformly) a pair with no active shift in any system of the block
        bool any = false;
        for (int h = 0; h < nsb; ++h)
            for (int u = 0; u < U; ++u)
                any = any || (steps_of(h) != 0 && s0 + u < nsh && st->sh[sys_of(h)][s0 + u].block_active);
        if (!any) continue;
        __syncthreads();   // the previous pair's coefficients have been read
        for (int e = threadIdx.x; e < nsb * U * (Q + 1); e += kBlock) {
            const int h = e / (U * (Q + 1)), r = e - h * U * (Q + 1);
            const int u = r / (Q + 1), l = r - u * (Q + 1);
            const int jj = sys_of(h);
            const int sh = s0 + u < nsh ? s0 + u : s0;   // the absent partner: any valid shift
            if (jj < a.nsys) {
                const BlockCoef& bc = coef[jj * kMaxShift + sh];
                cs[h][u][l] = l == 0 ? make_double2(bc.e, bc.c) : make_double2(bc.f[l], bc.d[l]);
            }
        }
        __syncthreads();
        bool act[U];
#pragma unroll
        for (int u = 0; u < U; ++u) act[u] = q != 0 && s0 + u < nsh && st->sh[j][s0 + u].block_active;
        if (!live || !(act[0] || act[1])) continue;
        double xr[U], xi[U], pr[U], pi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int sh = s0 + u;
            double2 xv = make_double2(0.0, 0.0);
            double p0r = rre[0], p0i = rim[0];
            if (act[u] && !first) {
                xv = X[j * a.x_sys + sh * a.x_shift + i];
                const double2 pv = P[((size_t)j * nsh + sh) * a.n + i];
                p0r = pv.x;
                p0i = pv.y;
            }
            const double2 ec = cs[hs][u][0];
            xr[u] = xv.x + ec.x * p0r;
            xi[u] = xv.y + ec.x * p0i;
            pr[u] = ec.y * p0r;
            pi[u] = ec.y * p0i;
        }
        // Each stored residual is widened once per pair of shifts, where it
        // is used, and the coefficients are read a few steps at a time: the
        // empty asms keep the compiler from widening the whole ring or
        // reading every coefficient up front, which would not fit the
        // registers.
        constexpr int kChunk = 2;
#pragma unroll
        for (int l0 = 1; l0 <= Q; l0 += kChunk) {
            // the previous chunk's sums are complete here, and no load of
            // this chunk moves above this point
            asm volatile("" : "+v"(xr[0]), "+v"(xi[0]), "+v"(pr[0]), "+v"(pi[0]), "+v"(xr[1]),
                         "+v"(xi[1]), "+v"(pr[1]), "+v"(pi[1])::"memory");
#pragma unroll
            for (int l = l0; l < l0 + kChunk && l <= Q; ++l) {
                RR re = rre[l], im = rim[l];
                if constexpr (std::is_same<RR, float>::value) asm volatile("" : "+v"(re), "+v"(im));
                const double dre = re, dim = im;
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const double2 fd = cs[hs][u][l];
                    xr[u] += fd.x * dre;
                    xi[u] += fd.x * dim;
                    pr[u] += fd.y * dre;
                    pi[u] += fd.y * dim;
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (!act[u]) continue;
            const int sh = s0 + u;
            X[j * a.x_sys + sh * a.x_shift + i] = make_double2(xr[u], xi[u]);
            if (st->sh[j][sh].active) P[((size_t)j * nsh + sh) * a.n + i] = make_double2(pr[u], pi[u]);
        }
    }
    if (!live) return;
    if (a.y) {
        // two-pass rational apply: residuals r(k0)..r(k0+q-1) of this block
        // (the host checks that this pass repeats the first one; the bound
        // keeps a mismatch from reading past the weights)
        const int k0 = st->sys[j].iters - q;
        const double* wj = a.w + (size_t)j * a.w_stride + k0;
        double2 yv = a.y[(size_t)j * a.n + i];
#pragma unroll
        for (int l = 0; l < Q; ++l)
            if (l < q && k0 >= 0 && (size_t)(k0 + l) < a.w_stride) {
                const double wl = wj[l];
                yv.x += wl * (double)rre[l];
                yv.y += wl * (double)rim[l];
            }
        a.y[(size_t)j * a.n + i] = yv;
    }
    // the last stored residual is r(k0) of the next block
#pragma unroll
    for (int l = 1; l <= Q; ++l)
        if (l == q) {
            VT v;
            v.x = rre[l];
            v.y = rim[l];
            a.ring[off] = v;
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

// ------------------------------------------------------------------ dot
// Re <a, b> (FP64) per system; block partials finished by k_finalize.
__global__ __launch_bounds__(kBlock) void k_dot(DotArgs a) {
    const int j = blockIdx.y;
    double d = 0.0;
    for (size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2; i < a.n;
         i += (size_t)gridDim.x * kBlock * 2) {
        Pair<double2> u, v;
        u.load(a.a[j], i);
        v.load(a.b[j], i);
        for (int k = 0; k < 2; ++k) d += u.re[k] * v.re[k] + u.im[k] * v.im[k];
    }
    reduce_store(d, 0.0, j, -1, a.partial);
}

// Re <a_j, b_j> of FP32 vectors with FP64 accumulation (the alpha numerator
// after a residual replacement).
__global__ __launch_bounds__(kBlock) void k_dot32(Dot32Args a) {
    const int j = blockIdx.y;
    double d = 0.0;
    for (size_t i = ((size_t)blockIdx.x * kBlock + threadIdx.x) * 2; i < a.n;
         i += (size_t)gridDim.x * kBlock * 2) {
        Pair<float2> u, v;
        load_sys(u, a.a[j], i, a.paired);
        load_sys(v, a.b[j], i, a.paired);
        for (int k = 0; k < 2; ++k)
            d += (double)u.re[k] * (double)v.re[k] + (double)u.im[k] * (double)v.im[k];
    }
    reduce_store(d, 0.0, j, -1, a.partial);
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

// ------------------------------------------------------------------ two-pass weights
// Two-pass rational apply.  x_i = sum_k c_i(k) r(k) over the steps k < N_i a
// shift took part in (the shifted recurrences of Sec. 4.3:
// x_i += a_i p_i, p_i' = zeta_i' r' + b_i p_i, p_i(0) = r(0)):
//   c_i(k) = zeta_i(k) G_i(k),  G_i(k) = a_i(k) + b_i(k) G_i(k+1),  G_i(N_i) = 0,
// with zeta_i, a_i = alpha zeta_i(k+1)/zeta_i(k), b_i = beta (zeta_i(k+1)/zeta_i(k))^2
// rebuilt from the recorded base alpha and beta by the recurrence the solve
// ran (shift_zeta_next).  One thread per (system, shift).
__global__ __launch_bounds__(kBlock) void k_two_pass_coef(TwoPassArgs a) {
    const SolverState* st = reinterpret_cast<const SolverState*>(a.state);
    const int nsh = st->nshift;
    const int p = threadIdx.x;
    if (p >= st->nsys * nsh) return;
    const int j = p / nsh, i = p % nsh;
    const ShiftScalars& h = st->sh[j][i];
    const int N = h.active ? st->sys[j].iters : h.conv_iter;
    const double* hj = a.hist + (size_t)j * a.hist_cap * 3;
    double* az = a.coef + (size_t)p * 3 * a.nmax;   // [a_i | b_i | zeta_i], each nmax
    double zeta = 1.0, zeta_prev = 1.0, alpha_prev = 1.0, beta_prev = 0.0;
    for (int k = 0; k < N; ++k) {
        const double alpha = hj[3 * k], beta = hj[3 * k + 1];
        const double zn = shift_zeta_next(zeta, zeta_prev, alpha, alpha_prev, beta_prev, h.off);
        const double ratio = zn / zeta;
        az[k] = alpha * ratio;
        az[a.nmax + k] = beta * ratio * ratio;
        az[2 * a.nmax + k] = zeta;
        zeta_prev = zeta;
        zeta = zn;
        alpha_prev = alpha;
        beta_prev = beta;
    }
    double G = 0.0;
    for (int k = N - 1; k >= 0; --k) {
        G = az[k] + az[a.nmax + k] * G;
        az[k] = az[2 * a.nmax + k] * G;   // c_i(k)
    }
    for (int k = N; k < a.nmax; ++k) az[k] = 0.0;
}

// w_j(k) = sum_i alpha_i c_ji(k), summed over i in order.
__global__ __launch_bounds__(kBlock) void k_two_pass_w(TwoPassArgs a) {
    const SolverState* st = reinterpret_cast<const SolverState*>(a.state);
    const int j = blockIdx.y, nsh = st->nshift;
    const int k = blockIdx.x * kBlock + threadIdx.x;
    if (k >= a.nmax) return;
    double w = 0.0;
    for (int i = 0; i < nsh; ++i) w += a.alpha[i] * a.coef[(size_t)(j * nsh + i) * 3 * a.nmax + k];
    a.w[(size_t)j * a.nmax + k] = w;
}

// ------------------------------------------------------------------ narrow
// y = x rounded to FP32 (round to nearest even), one complex number per thread
__global__ __launch_bounds__(kBlock) void k_narrow(NarrowArgs a) {
    const int j = blockIdx.y;
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= a.n) return;
    const double2 v = a.x[j][i];
    a.y[j][i << a.paired] = make_float2((float)v.x, (float)v.y);
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
// Paired FP32 sets run one block row per pair with the same number of blocks
// per row (and so of partial sums per system) as the unpaired kernels.
template <typename VT>
hipError_t launch_rupdate(const VecArgs<VT>& a, int nsys, hipStream_t s) {
    if constexpr (std::is_same<VT, float2>::value) {
        if (a.paired) {
            hipLaunchKernelGGL(k_rupdate_pair, red_grid(a.n, (nsys + 1) / 2), dim3(kBlock), 0, s, a);
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL(k_rupdate<VT>, red_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
template <typename VT>
hipError_t launch_pupdate(const VecArgs<VT>& a, int nsys, hipStream_t s) {
    // one extra block column: x = 0 runs the scalar recurrences
    if constexpr (std::is_same<VT, float2>::value) {
        if (a.paired) {
            const dim3 g(vec_blocks(a.n) + 1, (unsigned)((nsys + 1) / 2));
            hipLaunchKernelGGL(k_pupdate_pair, g, dim3(kBlock), 0, s, a);
            return hipGetLastError();
        }
    }
    const dim3 g(vec_blocks(a.n) + 1, (unsigned)nsys);
    hipLaunchKernelGGL(k_pupdate<VT>, g, dim3(kBlock), 0, s, a);
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
    const BlockCoef* coef = reinterpret_cast<const BlockCoef*>(a.coef);
    const int per = a.paired ? kBlock / 2 : kBlock;   // elements per block
    const dim3 g((unsigned)((a.n + per - 1) / per), (unsigned)(a.paired ? (nsys + 1) / 2 : nsys)),
        b(kBlock);
    // register arrays sized by the block length (coefficients beyond a
    // shift's last step are zero, so rounding up only adds idle terms); an
    // FP32 ring of 5 to 32 steps takes the 32-step form, the shortest that
    // keeps it in FP32 registers without spilling
    if (std::is_same<VT, float2>::value && qmax > 4 && qmax <= 32)
        hipLaunchKernelGGL((k_flush<VT, 32>), g, b, 0, s, a, coef);
    else if (qmax <= 4)
        hipLaunchKernelGGL((k_flush<VT, 4>), g, b, 0, s, a, coef);
    else if (qmax <= 16)
        hipLaunchKernelGGL((k_flush<VT, 16>), g, b, 0, s, a, coef);
    else if (qmax <= 20)
        hipLaunchKernelGGL((k_flush<VT, 20>), g, b, 0, s, a, coef);
    else if (qmax <= 25)
        hipLaunchKernelGGL((k_flush<VT, 25>), g, b, 0, s, a, coef);
    else if (qmax <= 32)
        hipLaunchKernelGGL((k_flush<VT, 32>), g, b, 0, s, a, coef);
    else
        hipLaunchKernelGGL((k_flush<VT, 50>), g, b, 0, s, a, coef);
    hipLaunchKernelGGL(k_flush_reset, dim3(1), dim3(kBlock), 0, s, a.state);
    return hipGetLastError();
}
hipError_t launch_combine(const CombineArgs& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_combine, vec_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_dot(const DotArgs& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_dot, red_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_dot32(const Dot32Args& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_dot32, red_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_add(const AddArgs& a, int nsys, hipStream_t s) {
    hipLaunchKernelGGL(k_add, vec_grid(a.n, nsys), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_two_pass_weights(const TwoPassArgs& a, int nsys, int nshift, hipStream_t s) {
    if (nsys * nshift > kBlock) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_two_pass_coef, dim3(1), dim3(kBlock), 0, s, a);
    const dim3 g((unsigned)((a.nmax + kBlock - 1) / kBlock), (unsigned)nsys);
    hipLaunchKernelGGL(k_two_pass_w, g, dim3(kBlock), 0, s, a);
    return hipGetLastError();
}
hipError_t launch_narrow(const NarrowArgs& a, int nsys, hipStream_t s) {
    const dim3 g((unsigned)((a.n + kBlock - 1) / kBlock), (unsigned)nsys);
    hipLaunchKernelGGL(k_narrow, g, dim3(kBlock), 0, s, a);
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
