// Self-energy diagonals of the static COHSEX approximation (Algorithm 3, steps 5-7).
//
// With W_s the screened interaction on the points of a pair set s (an N_mu x N_mu
// Hermitian matrix) and G(mu, nu) = sum_{i in set} psi_i(r_mu) conj(psi_i(r_nu)),
// eq. Hadamard turns the pair sum over i into
//   Sigma(n) = coef * sum_{mu, nu} conj(psi_n(r_mu)) (W_s (.) G)(mu, nu) psi_n(r_nu),
// the diagonal of Psi^H (W_s (.) G) Psi.  The product E = (W_s (.) G) Psi runs as a
// GEMM; these kernels form the Hadamard product and the column reductions.
#include "internal.h"

#include <algorithm>

namespace isdf {

namespace {

struct z2 { double re, im; };

__global__ __launch_bounds__(256) void mul_z_kernel(const z2* __restrict__ a, const z2* __restrict__ b,
                                                    z2* __restrict__ c, long count) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long k = (long)blockIdx.x * blockDim.x + threadIdx.x; k < count; k += stride) {
    const z2 x = a[k], y = b[k];
    c[k] = z2{x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re};
  }
}

// out[n] = coef * Re sum_mu conj(pm[n][mu]) e[mu][n]; one workgroup per band n,
// each thread a strided partial sum, then a fixed-order tree in LDS.
__global__ __launch_bounds__(256) void sigma_diag_kernel(const z2* __restrict__ pm, const z2* __restrict__ e,
                                                         int nmu, int ns, double coef, double* __restrict__ out) {
  __shared__ double red[256];
  const int n = blockIdx.x;
  double acc = 0.0;
  for (int mu = threadIdx.x; mu < nmu; mu += blockDim.x) {
    const z2 p = pm[(long)n * nmu + mu], v = e[(long)mu * ns + n];
    acc += p.re * v.re + p.im * v.im;
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = coef * red[0];
}

}  // namespace

hipError_t mul_z(const void* a, const void* b, void* c, long count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const long blocks = std::min<long>((count + 255) / 256, 4096);
  hipLaunchKernelGGL(mul_z_kernel, dim3((unsigned)blocks), dim3(256), 0, st, (const z2*)a, (const z2*)b, (z2*)c,
                     count);
  return hipGetLastError();
}

hipError_t sigma_diag(const void* pm, const void* e, int nmu, int ns, double coef, double* out, hipStream_t st) {
  if (ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(sigma_diag_kernel, dim3(ns), dim3(256), 0, st, (const z2*)pm, (const z2*)e, nmu, ns, coef,
                     out);
  return hipGetLastError();
}

}  // namespace isdf
