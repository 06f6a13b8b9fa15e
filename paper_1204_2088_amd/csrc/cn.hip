// cn.hip -- vector kernels of the Newton-Krylov solve of the Crank-Nicolson step
// (section 2: the diffusive part of eq. 3 is integrated implicitly).  The unknowns are
// the fields of phi^{n+1}; the host drives Newton's method with restarted GMRES on the
// finite-difference Jacobian, using these kernels for the residual assembly and the
// Krylov basis (dot products with fixed-order reductions, so runs are reproducible).
#include "device_common.h"

namespace hsf {

namespace {

constexpr int kVecBlocks = 512;   // blocks of the vector kernels (grid-stride)

// part[j * kVecBlocks + b] = block b's part of <V_j, x>, j = blockIdx.y
__global__ __launch_bounds__(kBlock) void k_dots(const double *__restrict__ V, long long n,
                                                 const double *__restrict__ x, double *__restrict__ part)
{
    const double *v = V + (long long)blockIdx.y * n;
    double acc = 0.0;
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)kVecBlocks * kBlock)
        acc += v[i] * x[i];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) part[(long long)blockIdx.y * kVecBlocks + blockIdx.x] = t;
}

// out[j] = sum of the kVecBlocks partials of dot j in a fixed order (one block per j)
__global__ __launch_bounds__(kBlock) void k_dots_final(const double *__restrict__ part, double *__restrict__ out)
{
    double acc = 0.0;
    for (int b = threadIdx.x; b < kVecBlocks; b += kBlock) acc += part[(long long)blockIdx.x * kVecBlocks + b];
    const double t = block_sum(acc);
    if (threadIdx.x == 0) out[blockIdx.x] = t;
}

// y += scale sum_j coef[j] V_j  (coef in device memory, k <= kMaxKrylov + 1)
__global__ __launch_bounds__(kBlock) void k_multi_axpy(double *__restrict__ y, const double *__restrict__ V, int k,
                                                       long long n, const double *__restrict__ coef, double scale)
{
    __shared__ double cs[kMaxKrylov + 1];
    for (int j = threadIdx.x; j < k; j += kBlock) cs[j] = scale * coef[j];
    __syncthreads();
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock) {
        double a = y[i];
        for (int j = 0; j < k; ++j) a = fma(cs[j], V[(long long)j * n + i], a);
        y[i] = a;
    }
}

// out = a x + b y (out may be x or y)
__global__ __launch_bounds__(kBlock) void k_lincomb(double *out, double a, const double *x, double b, const double *y,
                                                    long long n)
{
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        out[i] = a * x[i] + b * y[i];
}

// F = phi[w] - (half - phi[w]) - rhs, half = phi[w] + dt/2 B(phi[w], mu)
__global__ __launch_bounds__(kBlock) void k_cn_residual(double *__restrict__ F, const double *__restrict__ p,
                                                        const double *__restrict__ half,
                                                        const double *__restrict__ rhs, long long n)
{
    for (long long i = (long long)blockIdx.x * kBlock + threadIdx.x; i < n; i += (long long)gridDim.x * kBlock)
        F[i] = (p[i] - (half[i] - p[i])) - rhs[i];
}

}  // namespace

int vec_dot_blocks() { return kVecBlocks; }

void launch_dots(hipStream_t s, const double *V, int k, long long n, const double *x, double *part, double *out)
{
    hipLaunchKernelGGL(k_dots, dim3(kVecBlocks, k), dim3(kBlock), 0, s, V, n, x, part);
    hipLaunchKernelGGL(k_dots_final, dim3(k), dim3(kBlock), 0, s, (const double *)part, out);
}

void launch_multi_axpy(hipStream_t s, double *y, const double *V, int k, long long n, const double *coef,
                       double scale)
{
    hipLaunchKernelGGL(k_multi_axpy, dim3(kVecBlocks), dim3(kBlock), 0, s, y, V, k, n, coef, scale);
}

void launch_lincomb(hipStream_t s, double *out, double a, const double *x, double b, const double *y, long long n)
{
    hipLaunchKernelGGL(k_lincomb, dim3(kVecBlocks), dim3(kBlock), 0, s, out, a, x, b, y, n);
}

void launch_cn_residual(hipStream_t s, double *F, const double *p, const double *half, const double *rhs,
                        long long n)
{
    hipLaunchKernelGGL(k_cn_residual, dim3(kVecBlocks), dim3(kBlock), 0, s, F, p, half, rhs, n);
}

}  // namespace hsf
