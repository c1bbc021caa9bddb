// Launch arguments of the BLAS-1 kernels (blas.hip).
#pragma once

#include "common.h"

namespace rhmc {

// Generic per-system vector arguments; n = complex numbers per vector (3*Vh).
template <typename VT>
struct VecArgs {
    void* state;   // SolverState
    size_t n;
    const double2* b64[kMaxSys];
    VT* x[kMaxSys];
    VT* y[kMaxSys];
    VT* z[kMaxSys];
    double* partial;        // this kernel's block sums ([nsys][nblk]); read by k_pupdate
    int nblk;               // blocks per system of the kernel that wrote `partial`
    const double* part2;    // block sums of the A kernel (<p, A p>)
    int nblk2;
    int q;                  // step index inside the current block
    int paired;             // FP32 only: x, y, z are systems of paired sets (f32_offset);
                            // k_rupdate / k_pupdate then take one pair per block row
};

// Deferred update of the shifted solutions at a block boundary.
template <typename VT>
struct FlushArgs {
    void* state;
    const void* coef;       // BlockCoef [kMaxSys][kMaxShift]
    size_t n;
    int nshift;
    int nsys;
    VT* ring;               // stored base residuals: slot l (a set of nsys vectors) at
                            // ring + l*ring_slot; FP32 sets of two or more systems paired
    size_t ring_slot;
    int paired;
    double2* P;             // shifted directions [nsys][nshift][n], FP64 in every mode:
                            // rounding them is what limits a mixed solve's shifted
                            // true residuals, and they move only once per block
    double2* X;             // shifted solutions
    size_t x_sys, x_shift;  // element strides of X between systems / shifts
    // two-pass rational apply, second pass: y_j += sum_l w_j(k0+l) r(k0+l)
    // over the block's steps (y null: no accumulation)
    const double* w;        // [nsys][w_stride] weight of each base residual
    size_t w_stride;
    double2* y;             // [nsys][n]
};

// Weights of the two-pass rational apply (one block; state.h hist holds the
// first pass's per-step scalars).
struct TwoPassArgs {
    const void* state;      // SolverState after the first pass
    const double* hist;     // [nsys][hist_cap][3]: alpha, beta, <r', r'>
    int hist_cap;
    double* coef;           // [nsys][nshift][3 * nmax] scratch, then c_i(k) in the first nmax
    int nmax;               // largest step count of any system
    double alpha[kMaxShift];  // rational weights
    double* w;              // [nsys][nmax] output
};

struct CombineArgs {
    size_t n;
    int nterm;
    double alpha0;
    double alpha[kMaxShift];
    const double2* b[kMaxSys];
    const double2* x[kMaxSys];  // first of nterm vectors, x_stride elements apart
    size_t x_stride;
    double2* y[kMaxSys];
};

struct AddArgs {
    size_t n;
    const double2* x[kMaxSys];
    double2* y[kMaxSys];
};

// FP64 -> FP32 copy of up to kMaxSys vectors of n complex numbers (x and y
// must not overlap)
struct NarrowArgs {
    size_t n;
    const double2* x[kMaxSys];
    float2* y[kMaxSys];     // systems of an FP32 set
    int paired;             // y paired (element stride 2)
};

template <typename VT> hipError_t launch_start(const VecArgs<VT>& a, int nsys, hipStream_t s);
template <typename VT> hipError_t launch_rupdate(const VecArgs<VT>& a, int nsys, hipStream_t s);
template <typename VT> hipError_t launch_pupdate(const VecArgs<VT>& a, int nsys, hipStream_t s);
template <typename VT>
hipError_t launch_flush(const FlushArgs<VT>& a, int nsys, int qmax, hipStream_t s);
hipError_t launch_combine(const CombineArgs& a, int nsys, hipStream_t s);
// blocks along x of a vector kernel over n complex numbers (the partial-sum count)
int vec_blocks(size_t n);
// one-block kernel finishing block sums and running a FinalizeKind (state.h)
hipError_t launch_finalize(int kind, void* state, const double* partial, int nblk, int nrhs,
                           double* out_sums, hipStream_t s);
hipError_t launch_add(const AddArgs& a, int nsys, hipStream_t s);
hipError_t launch_narrow(const NarrowArgs& a, int nsys, hipStream_t s);
hipError_t launch_two_pass_weights(const TwoPassArgs& a, int nsys, int nshift, hipStream_t s);

// Re <a_j, b_j> per system, as block partials [nsys][vec_blocks(n)]
struct DotArgs {
    size_t n;
    const double2* a[kMaxSys];
    const double2* b[kMaxSys];
    double* partial;
};
hipError_t launch_dot(const DotArgs& a, int nsys, hipStream_t s);

// Re <a_j, b_j> of FP32 vectors (FP64 sums), same partial layout as DotArgs
struct Dot32Args {
    size_t n;
    const float2* a[kMaxSys];
    const float2* b[kMaxSys];
    double* partial;
    int paired;             // a and b are systems of paired sets (element stride 2)
};
hipError_t launch_dot32(const Dot32Args& a, int nsys, hipStream_t s);

}  // namespace rhmc
