// Cauchy-integral form of the core (Algorithm 2): M = f C Omega^{-1} C^H from
// resolvent-weighted orbital Grams on a contour around the empty-state energies.
//
// For node lambda_k (upper half of a contour symmetric about the real axis,
// quadrature weight w_k, nodes walked clockwise):
//   Av_k(mu, nu) = sum_i conj(psi_i(r_mu)) psi_i(r_nu) / (lambda_k - eps_i)
//   Ac_k(mu, nu) = sum_j psi_j(r_mu) conj(psi_j(r_nu)) / (lambda_k - eps_j)
//   S = sum_k w_k Av_k (.) Ac_k,      M = f / (2 pi i) (S - S^H)
// (the residue theorem gives 1 / (eps_i - eps_j) per pair; the lower half of
// the contour contributes -S^H).  The two Grams of a chunk of nodes are batched
// GEMMs over the scaled operands built here; S is accumulated in FP64 in a fixed
// node order.
#include "internal.h"
#include "common.h"

namespace isdf {

namespace {

// ops[kk][i][nu] = psi_i(r_nu) / (lambda_k - eps_i) (occupied rows) and
//                  conj(psi_j(r_nu)) / (lambda_k - eps_j) (empty rows), k = k0 + kk
// (T = double: complex128 out; T = float: complex64 out, for the single-precision engine)
template <typename T>
__global__ void cauchy_scale_kernel(const z64* __restrict__ pm, const double* __restrict__ e,
                                    const z64* __restrict__ lam, int nmu, int nv, int ns, int k0,
                                    cx<T>* __restrict__ ops) {
  const int nu = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y, kk = blockIdx.z;
  if (nu >= nmu) return;
  const z64 l = lam[k0 + kk];
  const double dr = l.re - e[n], di = l.im;
  const double s = 1.0 / (dr * dr + di * di);
  const z64 inv = {dr * s, -di * s};               // 1 / (lambda - eps_n)
  z64 p = pm[(long)n * nmu + nu];
  if (n >= nv) p.im = -p.im;
  ops[((long)kk * ns + n) * nmu + nu] = cx<T>{(T)(p.re * inv.re - p.im * inv.im), (T)(p.re * inv.im + p.im * inv.re)};
}

// s[mu][nu] += sum_kk w_k av[kk][mu][nu] ac[kk][mu][nu], in node order (products stored as cx<T>)
template <typename T>
__global__ void cauchy_accum_kernel(const cx<T>* __restrict__ av, const cx<T>* __restrict__ ac,
                                    const z64* __restrict__ w, int k0, int kc, long n2, z64* __restrict__ s) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n2) return;
  z64 acc = s[idx];
  for (int kk = 0; kk < kc; ++kk) {
    const z64 a = cvt<double>(av[kk * n2 + idx]), b = cvt<double>(ac[kk * n2 + idx]), wk = w[k0 + kk];
    const z64 j = {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
    acc.re += wk.re * j.re - wk.im * j.im;
    acc.im += wk.re * j.im + wk.im * j.re;
  }
  s[idx] = acc;
}

// m = f / (2 pi i) (s - s^H) = (f / (2 pi)) (-i) (s[mu][nu] - conj(s[nu][mu])); negm = -m (either optional)
__global__ void cauchy_finish_kernel(const z64* __restrict__ s, int n, double f, z64* __restrict__ m,
                                     z64* __restrict__ negm) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= n) return;
  const z64 a = s[(long)r * n + c], b = s[(long)c * n + r];
  const double dre = a.re - b.re, dim = a.im + b.im;   // s - conj(s^T)
  const double sc = f / (2.0 * M_PI);
  z64 v = {sc * dim, -sc * dre};                       // (-i) * (dre + i dim) * sc
  if (r == c) v.im = 0.0;                              // Hermitian: real diagonal
  if (m) m[(long)r * n + c] = v;
  if (negm) negm[(long)r * n + c] = z64{-v.re, -v.im};
}

}  // namespace

hipError_t cauchy_scale(const void* pm, const double* e, const void* lam, int nmu, int nv, int ns, int k0, int kc,
                        void* ops, bool ops32, hipStream_t st) {
  if (ops32)
    hipLaunchKernelGGL(cauchy_scale_kernel<float>, dim3(cdiv(nmu, 256), ns, kc), dim3(256), 0, st, (const z64*)pm,
                       e, (const z64*)lam, nmu, nv, ns, k0, (c32*)ops);
  else
    hipLaunchKernelGGL(cauchy_scale_kernel<double>, dim3(cdiv(nmu, 256), ns, kc), dim3(256), 0, st, (const z64*)pm,
                       e, (const z64*)lam, nmu, nv, ns, k0, (z64*)ops);
  return hipGetLastError();
}

hipError_t cauchy_accum(const void* av, const void* ac, bool prod32, const void* w, int k0, int kc, int nmu, void* s,
                        hipStream_t st) {
  const long n2 = (long)nmu * nmu;
  if (prod32)
    hipLaunchKernelGGL(cauchy_accum_kernel<float>, dim3(cdiv(n2, 256)), dim3(256), 0, st, (const c32*)av,
                       (const c32*)ac, (const z64*)w, k0, kc, n2, (z64*)s);
  else
    hipLaunchKernelGGL(cauchy_accum_kernel<double>, dim3(cdiv(n2, 256)), dim3(256), 0, st, (const z64*)av,
                       (const z64*)ac, (const z64*)w, k0, kc, n2, (z64*)s);
  return hipGetLastError();
}

hipError_t cauchy_finish(const void* s, int nmu, double f, void* m, void* negm, hipStream_t st) {
  hipLaunchKernelGGL(cauchy_finish_kernel, dim3(cdiv(nmu, 256), nmu), dim3(256), 0, st, (const z64*)s, nmu, f,
                     (z64*)m, (z64*)negm);
  return hipGetLastError();
}

}  // namespace isdf
