// Device kernels of the hand-written adjoint of L = Re tr(W eps~^{-1}) (FP64).
//
// The backward pass runs the forward's steps in reverse: the SMW step, U = X S^{-1},
// the pruned DFT (its adjoint here: the NG-list rows scattered back through the
// z, y and x stages with conjugated twiddles), the Hadamard pair products of the
// ISDF fit, the Hadamard Grams of S, and the core M = f C diag(w) C^H.  Every
// reduction is a fixed-order loop in one thread (no atomics), so the gradients
// are bit-reproducible.
#include "internal.h"
#include "common.h"

namespace isdf {

namespace {

__device__ __forceinline__ z64 zmul(z64 a, z64 b) { return z64{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ z64 zcmul(z64 a, z64 b) { return z64{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re}; }  // conj(a) b

// out = conj(x) * y
__global__ void conj_mul_kernel(const z64* __restrict__ x, const z64* __restrict__ y, z64* __restrict__ out, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = zcmul(x[i], y[i]);
}

// Backward of z = conj(p) * q:  p <- conj(g) * q,  q <- g * p (in place, element by element)
__global__ void pair_grad_kernel(const z64* __restrict__ g, z64* __restrict__ p, z64* __restrict__ q, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const z64 gi = g[i], pi = p[i], qi = q[i];
  p[i] = zcmul(gi, qi);
  q[i] = zmul(gi, pi);
}

// h[m][n] = g[m][n] + conj(g[n][m])
__global__ void herm_plus_kernel(const z64* __restrict__ g, z64* __restrict__ h, int n) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= n) return;
  const z64 a = g[(long)r * n + c], b = g[(long)c * n + r];
  h[(long)r * n + c] = z64{a.re + b.re, a.im - b.im};
}

// out[m][v] = src[m * ld + idx[v]]
__global__ void gather_cols_kernel(const z64* __restrict__ src, long ld, const int* __restrict__ idx, int nv,
                                   z64* __restrict__ out) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x, m = blockIdx.y;
  if (v < nv) out[(long)m * nv + v] = src[(long)m * ld + idx[v]];
}

// z stage: t2b[mu][d][z] = sum_{g in d} conj(twz[c_g][z]) sqrtv[g] gb[g][mu] (gb row stride ldg)
__global__ void adj_z_kernel(long ldg, int nd, int n2, const int* __restrict__ off, const int* __restrict__ list,
                             const int* __restrict__ g_cz, const z64* __restrict__ twz,
                             const double* __restrict__ sqrtv, const z64* __restrict__ gb, z64* __restrict__ t2b) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  if (t >= nd * n2) return;
  const int d = t / n2, z = t % n2;
  z64 acc = {0.0, 0.0};
  for (int e = off[d]; e < off[d + 1]; ++e) {
    const int g = list[e];
    const z64 v = gb[(long)g * ldg + mu];
    const z64 tw = twz[(long)g_cz[g] * n2 + z];
    const z64 p = zcmul(tw, v);
    acc.re += sqrtv[g] * p.re;
    acc.im += sqrtv[g] * p.im;
  }
  t2b[((long)mu * nd + d) * n2 + z] = acc;
}

// y stage: t1b[mu][z][y][a] = sum_{d with a_d = a} conj(twy[b_d][y]) t2b[mu][d][z]
__global__ void adj_y_kernel(int nd, int n1, int n2, int kx, const int* __restrict__ off,
                             const int* __restrict__ list, const int* __restrict__ d_by,
                             const z64* __restrict__ twy, const z64* __restrict__ t2b, z64* __restrict__ t1b) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  if (t >= (long)kx * n1 * n2) return;
  const int a = (int)(t % kx), y = (int)((t / kx) % n1), z = (int)(t / ((long)kx * n1));
  z64 acc = {0.0, 0.0};
  for (int e = off[a]; e < off[a + 1]; ++e) {
    const int d = list[e];
    const z64 p = zcmul(twy[(long)d_by[d] * n1 + y], t2b[((long)mu * nd + d) * n2 + z]);
    acc.re += p.re;
    acc.im += p.im;
  }
  t1b[(((long)mu * n2 + z) * n1 + y) * kx + a] = acc;
}

// x stage: gz[mu][r] = sum_a conj(twx[a][x]) t1b[mu][z][y][a], r = x + n0 (y + n1 z)
__global__ void adj_x_kernel(int n0, int n1, int n2, int kx, const z64* __restrict__ twx,
                             const z64* __restrict__ t1b, z64* __restrict__ gz) {
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  const long nr = (long)n0 * n1 * n2;
  if (r >= nr) return;
  const int x = (int)(r % n0);
  const long yz = r / n0;   // y + n1 z
  const z64* src = t1b + ((long)mu * n2 * n1 + yz) * kx;
  z64 acc = {0.0, 0.0};
  for (int a = 0; a < kx; ++a) {
    const z64 p = zcmul(twx[(long)a * n0 + x], src[a]);
    acc.re += p.re;
    acc.im += p.im;
  }
  gz[(long)mu * nr + r] = acc;
}

// cb[ii][v][j] = conj(a[i0 + ii][v]) b[j][v]   (a = pm rows 0..nv-1, b = rows nv..)
__global__ void core_pairs_kernel(const z64* __restrict__ pm, int nmu, int nv, int nc, int i0, z64* __restrict__ cb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int v = blockIdx.y, ii = blockIdx.z;
  if (j >= nc) return;
  cb[((long)ii * nmu + v) * nc + j] = zcmul(pm[(long)(i0 + ii) * nmu + v], pm[(long)(nv + j) * nmu + v]);
}

// G_a(i, mu) += 2 f sum_j w_ij b_j(mu) conj(U_i(mu, j))   (one thread per (ii, mu))
__global__ void core_grad_a_kernel(const z64* __restrict__ ub, const z64* __restrict__ pm, const double* __restrict__ w,
                                   int nmu, int nv, int nc, int i0, int nb, double f, z64* __restrict__ ga) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x, ii = blockIdx.y;
  if (mu >= nmu || ii >= nb) return;
  const int i = i0 + ii;
  const z64* u = ub + ((long)ii * nmu + mu) * nc;
  z64 acc = {0.0, 0.0};
  for (int j = 0; j < nc; ++j) {
    const z64 p = zcmul(u[j], pm[(long)(nv + j) * nmu + mu]);   // conj(U) b
    const double wij = w[(long)i * nc + j];
    acc.re += wij * p.re;
    acc.im += wij * p.im;
  }
  z64& o = ga[(long)i * nmu + mu];
  o.re += 2.0 * f * acc.re;
  o.im += 2.0 * f * acc.im;
}

// q[i][j] = f sum_mu conj(b_j(mu)) a_i(mu) U_i(mu, j)   (one thread per (ii, j))
__global__ void core_grad_q_kernel(const z64* __restrict__ ub, const z64* __restrict__ pm, int nmu, int nv, int nc,
                                   int i0, int nb, double f, z64* __restrict__ q) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, ii = blockIdx.y;
  if (j >= nc || ii >= nb) return;
  const int i = i0 + ii;
  z64 acc = {0.0, 0.0};
  for (int mu = 0; mu < nmu; ++mu) {
    const z64 ab = zcmul(pm[(long)(nv + j) * nmu + mu], pm[(long)i * nmu + mu]);   // conj(b) a
    const z64 p = zmul(ab, ub[((long)ii * nmu + mu) * nc + j]);
    acc.re += p.re;
    acc.im += p.im;
  }
  q[(long)i * nc + j] = z64{f * acc.re, f * acc.im};
}

// G_b(j, mu) += 2 f sum_{ii} w_ij a_i(mu) U_i(mu, j)   (one thread per (j, mu); batches in order)
__global__ void core_grad_b_kernel(const z64* __restrict__ ub, const z64* __restrict__ pm, const double* __restrict__ w,
                                   int nmu, int nv, int nc, int i0, int nb, double f, z64* __restrict__ gb) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x, mu = blockIdx.y;
  if (j >= nc) return;
  z64 acc = {0.0, 0.0};
  for (int ii = 0; ii < nb; ++ii) {
    const int i = i0 + ii;
    const z64 p = zmul(pm[(long)i * nmu + mu], ub[((long)ii * nmu + mu) * nc + j]);
    const double wij = w[(long)i * nc + j];
    acc.re += wij * p.re;
    acc.im += wij * p.im;
  }
  z64& o = gb[(long)j * nmu + mu];
  o.re += 2.0 * f * acc.re;
  o.im += 2.0 * f * acc.im;
}

// dL/d eps: ge[i] = sum_j Re q_ij w'_ij, ge[nv + j] = -sum_i Re q_ij w'_ij,
// w'_ij = (omega^2 - D^2) / (D^2 + omega^2)^2, D = eps_i - eps_{nv + j}
__global__ void energy_grad_kernel(const z64* __restrict__ q, const double* __restrict__ e, int nv, int nc,
                                   double omega, double* __restrict__ ge) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= nv + nc) return;
  const double o2 = omega * omega;
  double acc = 0.0;
  if (n < nv) {
    for (int j = 0; j < nc; ++j) {
      const double d = e[n] - e[nv + j], s = d * d + o2;
      acc += q[(long)n * nc + j].re * (o2 - d * d) / (s * s);
    }
  } else {
    const int j = n - nv;
    for (int i = 0; i < nv; ++i) {
      const double d = e[i] - e[nv + j], s = d * d + o2;
      acc -= q[(long)i * nc + j].re * (o2 - d * d) / (s * s);
    }
  }
  ge[n] = acc;
}

// out[0] = Re tr(w) over its ng x ng block (row stride ldw) + Re tr(p) (n x n): one workgroup, fixed tree
__global__ __launch_bounds__(256) void loss_kernel(const z64* __restrict__ w, int ng, long ldw, const z64* __restrict__ p,
                                                   int n, double* __restrict__ out) {
  __shared__ double s[256];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int i = t; i < ng; i += 256) acc += w[(long)i * ldw + i].re;
  for (int i = t; i < n; i += 256) acc += p[(long)i * n + i].re;
  s[t] = acc;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if (t < k) s[t] += s[t + k];
    __syncthreads();
  }
  if (t == 0) out[0] = s[0];
}

}  // namespace

hipError_t adj_conj_mul(const void* x, const void* y, void* out, long n, hipStream_t st) {
  hipLaunchKernelGGL(conj_mul_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, (const z64*)x, (const z64*)y, (z64*)out, n);
  return hipGetLastError();
}

hipError_t adj_pair_grad(const void* g, void* p, void* q, long n, hipStream_t st) {
  hipLaunchKernelGGL(pair_grad_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, (const z64*)g, (z64*)p, (z64*)q, n);
  return hipGetLastError();
}

hipError_t adj_herm_plus(const void* g, void* h, int n, hipStream_t st) {
  hipLaunchKernelGGL(herm_plus_kernel, dim3(cdiv(n, 256), n), dim3(256), 0, st, (const z64*)g, (z64*)h, n);
  return hipGetLastError();
}

hipError_t adj_gather_cols(const void* src, long ld, const int* idx, int nv, int rows, void* out, hipStream_t st) {
  hipLaunchKernelGGL(gather_cols_kernel, dim3(cdiv(nv, 256), rows), dim3(256), 0, st, (const z64*)src, ld, idx, nv,
                     (z64*)out);
  return hipGetLastError();
}

hipError_t adj_dft(const AdjDft& a, const void* gbar, void* t2b, void* t1b, void* gz, hipStream_t st) {
  hipLaunchKernelGGL(adj_z_kernel, dim3(cdiv((long)a.nd * a.n2, 256), a.nmu), dim3(256), 0, st, a.ldg, a.nd, a.n2,
                     a.gd_off, a.gd_list, a.g_cz, (const z64*)a.twz, a.sqrtv, (const z64*)gbar, (z64*)t2b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_y_kernel, dim3(cdiv((long)a.kx * a.n1 * a.n2, 256), a.nmu), dim3(256), 0, st, a.nd, a.n1,
                     a.n2, a.kx, a.da_off, a.da_list, a.d_by, (const z64*)a.twy, (const z64*)t2b, (z64*)t1b);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(adj_x_kernel, dim3(cdiv((long)a.n0 * a.n1 * a.n2, 256), a.nmu), dim3(256), 0, st, a.n0, a.n1,
                     a.n2, a.kx, (const z64*)a.twx, (const z64*)t1b, (z64*)gz);
  return hipGetLastError();
}

hipError_t adj_core_pairs(const void* pm, int nmu, int nv, int nc, int i0, int nb, void* cb, hipStream_t st) {
  hipLaunchKernelGGL(core_pairs_kernel, dim3(cdiv(nc, 256), nmu, nb), dim3(256), 0, st, (const z64*)pm, nmu, nv, nc,
                     i0, (z64*)cb);
  return hipGetLastError();
}

hipError_t adj_core_grads(const void* ub, const void* pm, const double* w, int nmu, int nv, int nc, int i0, int nb,
                          double f, void* ga, void* q, void* gb, hipStream_t st) {
  hipLaunchKernelGGL(core_grad_a_kernel, dim3(cdiv(nmu, 256), nb), dim3(256), 0, st, (const z64*)ub, (const z64*)pm,
                     w, nmu, nv, nc, i0, nb, f, (z64*)ga);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(core_grad_q_kernel, dim3(cdiv(nc, 256), nb), dim3(256), 0, st, (const z64*)ub, (const z64*)pm,
                     nmu, nv, nc, i0, nb, f, (z64*)q);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(core_grad_b_kernel, dim3(cdiv(nc, 256), nmu), dim3(256), 0, st, (const z64*)ub, (const z64*)pm,
                     w, nmu, nv, nc, i0, nb, f, (z64*)gb);
  return hipGetLastError();
}

hipError_t adj_energy_grad(const void* q, const double* e, int nv, int nc, double omega, double* ge, hipStream_t st) {
  hipLaunchKernelGGL(energy_grad_kernel, dim3(cdiv(nv + nc, 256)), dim3(256), 0, st, (const z64*)q, e, nv, nc, omega,
                     ge);
  return hipGetLastError();
}

hipError_t adj_loss(const void* w, int ng, long ldw, const void* p, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, st, (const z64*)w, ng, ldw, (const z64*)p, n, out);
  return hipGetLastError();
}

}  // namespace isdf
