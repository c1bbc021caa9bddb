// FP64 3x3 complex matrix helpers and the su(3) algebra of the momenta
// (Sec. 2.1): H = sum_a omega^a T^a with T^a = lambda^a / 2, traceless
// Hermitian, one per link.
#pragma once

#include "dslash_kernel.h"

namespace rhmc {

typedef Link<double> Mat3;

#if defined(__HIPCC__)
__device__ __forceinline__ void mat_zero(Mat3& a) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) a.re[i][j] = a.im[i][j] = 0.0;
}

__device__ __forceinline__ void mat_identity(Mat3& a) {
    mat_zero(a);
    a.re[0][0] = a.re[1][1] = a.re[2][2] = 1.0;
}

// c = a b (DA, DB select a^dagger, b^dagger); ACC: c += a b.  Each real and
// imaginary part is one chain of fused multiply-adds over k (four per complex
// product instead of a multiply, a fused multiply-add and an add).  c must
// not alias a or b.
template <bool DA, bool DB, bool ACC = false>
__device__ __forceinline__ void mat_mul(const Mat3& a, const Mat3& b, Mat3& c) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            double sr = ACC ? c.re[i][j] : 0.0, si = ACC ? c.im[i][j] : 0.0;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double ar = DA ? a.re[k][i] : a.re[i][k];
                const double ai = DA ? -a.im[k][i] : a.im[i][k];
                const double br = DB ? b.re[j][k] : b.re[k][j];
                const double bi = DB ? -b.im[j][k] : b.im[k][j];
                if (!ACC && k == 0) {
                    sr = ar * br;
                    si = ar * bi;
                } else {
                    sr = __builtin_fma(ar, br, sr);
                    si = __builtin_fma(ar, bi, si);
                }
                sr = __builtin_fma(-ai, bi, sr);
                si = __builtin_fma(ai, br, si);
            }
            c.re[i][j] = sr;
            c.im[i][j] = si;
        }
}

__device__ __forceinline__ void mat_add(Mat3& a, const Mat3& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            a.re[i][j] += b.re[i][j];
            a.im[i][j] += b.im[i][j];
        }
}

// Re Tr(a b^dagger) = sum_ij Re(a_ij conj(b_ij))
__device__ __forceinline__ double re_tr_mul_dagger(const Mat3& a, const Mat3& b) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) s += a.re[i][j] * b.re[i][j] + a.im[i][j] * b.im[i][j];
    return s;
}

// c^a = scale * i Tr(T^a TA(X)), TA the traceless anti-Hermitian part.  The
// trace part drops out (T^a is traceless), so with A = (X - X^dagger)/2 and
// h = i A (Hermitian) c^a = scale * Tr(T^a h), written out entry by entry.
__device__ __forceinline__ void algebra_coef(const Mat3& X, double scale, double c[8]) {
    const double k = 0.5 * scale;
    c[0] = -k * (X.im[0][1] + X.im[1][0]);
    c[1] = -k * (X.re[0][1] - X.re[1][0]);
    c[2] = k * (X.im[1][1] - X.im[0][0]);
    c[3] = -k * (X.im[0][2] + X.im[2][0]);
    c[4] = -k * (X.re[0][2] - X.re[2][0]);
    c[5] = -k * (X.im[1][2] + X.im[2][1]);
    c[6] = -k * (X.re[1][2] - X.re[2][1]);
    c[7] = k * (2.0 * X.im[2][2] - X.im[0][0] - X.im[1][1]) * 0.57735026918962576;   // 1/sqrt(3)
}

// H = sum_a omega^a T^a
__device__ __forceinline__ void algebra_matrix(const double w[8], Mat3& H) {
    const double s3 = 0.57735026918962576 * w[7];   // omega^8 / sqrt(3)
    H.re[0][0] = 0.5 * (w[2] + s3);
    H.re[1][1] = 0.5 * (s3 - w[2]);
    H.re[2][2] = -s3;
    H.im[0][0] = H.im[1][1] = H.im[2][2] = 0.0;
    H.re[0][1] = 0.5 * w[0];  H.im[0][1] = -0.5 * w[1];
    H.re[1][0] = 0.5 * w[0];  H.im[1][0] = 0.5 * w[1];
    H.re[0][2] = 0.5 * w[3];  H.im[0][2] = -0.5 * w[4];
    H.re[2][0] = 0.5 * w[3];  H.im[2][0] = 0.5 * w[4];
    H.re[1][2] = 0.5 * w[5];  H.im[1][2] = -0.5 * w[6];
    H.re[2][1] = 0.5 * w[5];  H.im[2][1] = 0.5 * w[6];
}
#endif  // __HIPCC__

}  // namespace rhmc
