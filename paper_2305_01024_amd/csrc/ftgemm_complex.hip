// ftgemm_complex.hip -- the data movement of the double-complex FT-GEMM
// (ftgemm_run_z64): the binary64 FT kernels run it as two real products.
//
// With A = Ar + i Ai and B = Br + i Bi (column-major, (re, im) pairs), and
// the inner index of each complex product split into two real ones,
//   Re(A B) = A' B'   with A'[i, 2p] = Ar[i, p],  A'[i, 2p + 1] = -Ai[i, p],
//   Im(A B) = A'' B'  with A''[i, 2p] = Ai[i, p], A''[i, 2p + 1] =  Ar[i, p],
// and B'[2p, j] = Br[p, j], B'[2p + 1, j] = Bi[p, j], which is B's own storage
// read as a real 2k x n matrix with leading dimension 2 ldb.  The checksum
// relations of the two real products are the real and imaginary parts of the
// complex ones (e^T A' = [Re e^T A, -Im e^T A] interleaved, B' e = B e
// interleaved), and a k-step of 2 ku real indices is a k-step of ku complex
// ones, so each component is checked, located and corrected on its own at
// the same check steps.  zrepack writes A' and A''; zepilogue applies the
// complex alpha and beta to the two real accumulators.
#include "ftgemm_internal.h"

namespace ftgemm_impl {
namespace {

// A (m x k complex, lda) -> A' and A'' (m x 2k real, leading dimension m)
__global__ void zrepack_kernel(const double* A, int64_t lda, int32_t M, int32_t K, double* Ap, double* App) {
    const int64_t total = (int64_t)M * K;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x % M, p = x / M;
        const double2 a = *reinterpret_cast<const double2*>(A + 2 * (i + p * lda));
        Ap[i + (2 * p) * (int64_t)M] = a.x;
        Ap[i + (2 * p + 1) * (int64_t)M] = -a.y;
        App[i + (2 * p) * (int64_t)M] = a.y;
        App[i + (2 * p + 1) * (int64_t)M] = a.x;
    }
}

// C = alpha (Pr + i Pi) + beta C (complex; beta == 0: C is not read)
__global__ void zepilogue_kernel(double* C, int64_t ldc, int32_t M, int32_t N, const double* Pr, const double* Pi,
                                 double ar, double ai, double br, double bi) {
    const int64_t total = (int64_t)M * N;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x % M, j = x / M;
        const double pr = Pr[x], pi = Pi[x];
        double2* c = reinterpret_cast<double2*>(C + 2 * (i + j * ldc));
        double2 v;
        v.x = ar * pr - ai * pi;
        v.y = ar * pi + ai * pr;
        if (br != 0.0 || bi != 0.0) {
            const double2 c0 = *c;
            v.x += br * c0.x - bi * c0.y;
            v.y += br * c0.y + bi * c0.x;
        }
        *c = v;
    }
}

// C = beta C (complex; beta == 0 writes zeros without reading C)
__global__ void zscale_kernel(double* C, int64_t ldc, int32_t M, int32_t N, double br, double bi) {
    const int64_t total = (int64_t)M * N;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < total; x += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = x % M, j = x / M;
        double2* c = reinterpret_cast<double2*>(C + 2 * (i + j * ldc));
        double2 v = {0.0, 0.0};
        if (br != 0.0 || bi != 0.0) {
            const double2 c0 = *c;
            v.x = br * c0.x - bi * c0.y;
            v.y = br * c0.y + bi * c0.x;
        }
        *c = v;
    }
}

unsigned grid_for(int64_t total) {
    const int64_t b = (total + 255) / 256;
    return (unsigned)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

hipError_t launch_zrepack(const double* A, int64_t lda, int32_t M, int32_t K, double* Ap, double* App,
                          hipStream_t s) {
    hipLaunchKernelGGL(zrepack_kernel, dim3(grid_for((int64_t)M * K)), dim3(256), 0, s, A, lda, M, K, Ap, App);
    return hipGetLastError();
}

hipError_t launch_zepilogue(double* C, int64_t ldc, int32_t M, int32_t N, const double* Pr, const double* Pi,
                            const double* alpha, const double* beta, hipStream_t s) {
    hipLaunchKernelGGL(zepilogue_kernel, dim3(grid_for((int64_t)M * N)), dim3(256), 0, s, C, ldc, M, N, Pr, Pi,
                       alpha[0], alpha[1], beta[0], beta[1]);
    return hipGetLastError();
}

hipError_t launch_zscale(double* C, int64_t ldc, int32_t M, int32_t N, const double* beta, hipStream_t s) {
    hipLaunchKernelGGL(zscale_kernel, dim3(grid_for((int64_t)M * N)), dim3(256), 0, s, C, ldc, M, N, beta[0],
                       beta[1]);
    return hipGetLastError();
}

}  // namespace ftgemm_impl
