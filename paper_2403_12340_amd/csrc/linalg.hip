// FP64 dense algebra on the N_mu x N_mu core (row-major complex128, ld = n).
//
//   potrf          blocked right-looking Cholesky A = L L^H (panel width 32):
//                  one kernel factors the diagonal block in LDS, inverts it and
//                  forms the sub-diagonal panel L_ik = A_ik L_kk^{-H}; the
//                  trailing update is an MFMA GEMM on the lower tiles.
//   sweep_inverse  blocked Gauss-Jordan sweep of a Hermitian positive definite
//                  matrix, A <- -A^{-1}: per 32-wide pivot block, one kernel
//                  inverts the pivot block and forms the row panel R = P A_k:,
//                  then one MFMA GEMM applies A_ij -= A_ik P A_kj to the whole
//                  matrix with the pivot row/column taken from R.
// A non-positive or non-finite pivot sets bit 0 of *status (ISDF_E_NOT_PD).
#include "internal.h"
#include "tile.h"

#include <cmath>

namespace isdf {

constexpr int NB = 32;

__device__ __forceinline__ z64 zdiv(z64 a, z64 b) {
  const double d = b.re * b.re + b.im * b.im;
  return z64{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

__global__ __launch_bounds__(256) void potrf_panel_kernel(int n, z64* a, int k0, int kn, int* status) {
  __shared__ z64 D[NB][NB + 1];
  __shared__ z64 X[NB][NB + 1];
  __shared__ z64 P[NB][NB + 1];
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kn * kn; idx += 256) {
    const int r = idx / kn, c = idx % kn;
    D[r][c] = (r >= c) ? a[(long)(k0 + r) * n + k0 + c] : z64{0.0, 0.0};
  }
  __syncthreads();
  for (int c = 0; c < kn; ++c) {
    if (tid == 0) {
      double d = D[c][c].re;
      if (!(d > 0.0) || !isfinite(d)) {
        atomicOr(status, 1);
        d = 1.0;
      }
      D[c][c] = z64{sqrt(d), 0.0};
    }
    __syncthreads();
    const double piv = D[c][c].re;
    for (int r = c + 1 + tid; r < kn; r += 256) D[r][c] = z64{D[r][c].re / piv, D[r][c].im / piv};
    __syncthreads();
    const int m = kn - c - 1;
    for (int idx = tid; idx < m * m; idx += 256) {
      const int r = c + 1 + idx / m, s = c + 1 + idx % m;
      if (s <= r) {
        const z64 x = cmul(D[r][c], cconj(D[s][c]));
        D[r][s].re -= x.re;
        D[r][s].im -= x.im;
      }
    }
    __syncthreads();
  }
  // X = L_kk^{-1}, one column per thread (forward substitution)
  if (tid < kn) {
    const int col = tid;
    for (int r = 0; r < kn; ++r) {
      if (r < col) { X[r][col] = z64{0.0, 0.0}; continue; }
      z64 s = (r == col) ? z64{1.0, 0.0} : z64{0.0, 0.0};
      for (int t = col; t < r; ++t) {
        const z64 x = cmul(D[r][t], X[t][col]);
        s.re -= x.re;
        s.im -= x.im;
      }
      X[r][col] = zdiv(s, D[r][r]);
    }
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    for (int idx = tid; idx < kn * kn; idx += 256) {
      const int r = idx / kn, c = idx % kn;
      a[(long)(k0 + r) * n + k0 + c] = (r >= c) ? D[r][c] : z64{0.0, 0.0};
    }
    // strict upper part of this block row right of the diagonal block
    const int w = n - k0 - kn;
    for (long idx = tid; idx < (long)kn * w; idx += 256) {
      const int r = (int)(idx / w), c = (int)(idx % w);
      a[(long)(k0 + r) * n + k0 + kn + c] = z64{0.0, 0.0};
    }
    return;
  }
  const int rb0 = k0 + kn + (blockIdx.x - 1) * NB;
  const int nr = min(NB, n - rb0);
  if (nr <= 0) return;
  for (int idx = tid; idx < nr * kn; idx += 256) {
    const int r = idx / kn, c = idx % kn;
    P[r][c] = a[(long)(rb0 + r) * n + k0 + c];
  }
  __syncthreads();
  // L_ik = A_ik X^H
  for (int idx = tid; idx < nr * kn; idx += 256) {
    const int r = idx / kn, c = idx % kn;
    z64 s{0.0, 0.0};
    for (int t = 0; t <= c; ++t) {
      const z64 x = cmul(P[r][t], cconj(X[c][t]));
      s.re += x.re;
      s.im += x.im;
    }
    a[(long)(rb0 + r) * n + k0 + c] = s;
  }
}

hipError_t potrf(int n, void* a, void* scratch, int* status, hipStream_t st) {
  (void)scratch;
  z64* A = (z64*)a;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kn = min(NB, n - k0);
    const int rest = n - k0 - kn;
    const int nblk = 1 + (rest + NB - 1) / NB;
    hipLaunchKernelGGL(potrf_panel_kernel, dim3(nblk), dim3(256), 0, st, n, A, k0, kn, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (rest > 0) {
      GemmDesc d;
      d.M = d.N = rest;
      d.K = kn;
      d.A = A + (long)(k0 + kn) * n + k0; d.sam = n; d.sak = 1;
      d.B = A + (long)(k0 + kn) * n + k0; d.sbk = 1; d.sbn = n; d.conjB = true;
      d.C = A + (long)(k0 + kn) * n + k0 + kn; d.ldc = n;
      d.alpha = -1.0; d.beta = 1.0; d.herm = true;
      e = gemm(P64, d, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void sweep_panel_kernel(int n, const z64* a, int k0, int kn, z64* R,
                                                          z64* Old, int* status) {
  __shared__ z64 W[NB][NB + 1];
  __shared__ z64 colp[NB];
  __shared__ z64 Pan[NB][64 + 1];
  const int tid = threadIdx.x;
  const int c0 = blockIdx.x * 64;
  for (int idx = tid; idx < kn * kn; idx += 256) {
    const int r = idx / kn, c = idx % kn;
    W[r][c] = a[(long)(k0 + r) * n + k0 + c];
  }
  __syncthreads();
  // in-place Gauss-Jordan inverse of the pivot block (Hermitian positive definite: no pivoting)
  for (int p = 0; p < kn; ++p) {
    const z64 piv = W[p][p];
    bool bad = !(piv.re > 0.0) || !isfinite(piv.re) || !isfinite(piv.im);
    const z64 d = bad ? z64{1.0, 0.0} : zdiv(z64{1.0, 0.0}, piv);
    if (bad && tid == 0) atomicOr(status, 1);
    __syncthreads();
    if (tid < kn) {
      colp[tid] = W[tid][p];
      W[p][tid] = (tid == p) ? d : cmul(W[p][tid], d);
    }
    __syncthreads();
    for (int idx = tid; idx < kn * kn; idx += 256) {
      const int r = idx / kn, j = idx % kn;
      if (r == p) continue;
      const z64 base = (j == p) ? z64{0.0, 0.0} : W[r][j];
      const z64 x = cmul(colp[r], W[p][j]);
      W[r][j] = z64{base.re - x.re, base.im - x.im};
    }
    __syncthreads();
  }
  const int nc = min(64, n - c0);
  for (int idx = tid; idx < kn * nc; idx += 256) {
    const int t = idx / nc, c = idx % nc;
    Pan[t][c] = a[(long)(k0 + t) * n + c0 + c];
  }
  __syncthreads();
  for (int idx = tid; idx < kn * nc; idx += 256) {
    const int t = idx / nc, c = idx % nc;
    const int gc = c0 + c;
    Old[(long)t * n + gc] = Pan[t][c];
    z64 s{0.0, 0.0};
    if (gc >= k0 && gc < k0 + kn) {
      s = z64{-W[t][gc - k0].re, -W[t][gc - k0].im};
    } else {
      for (int u = 0; u < kn; ++u) {
        const z64 x = cmul(W[t][u], Pan[u][c]);
        s.re += x.re;
        s.im += x.im;
      }
    }
    R[(long)t * n + gc] = s;
  }
}

size_t linalg_scratch_bytes(int n) { return (size_t)2 * NB * n * sizeof(z64); }

hipError_t sweep_inverse(int n, void* a, void* scratch, int* status, hipStream_t st) {
  z64* A = (z64*)a;
  z64* R = (z64*)scratch;
  z64* Old = R + (long)NB * n;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kn = min(NB, n - k0);
    hipLaunchKernelGGL(sweep_panel_kernel, dim3(cdiv(n, 64)), dim3(256), 0, st, n, (const z64*)A, k0,
                       kn, R, Old, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    GemmDesc d;
    d.M = d.N = n;
    d.K = kn;
    d.A = Old; d.sam = 1; d.sak = n; d.conjA = true;
    d.B = R; d.sbk = n; d.sbn = 1;
    d.C = A; d.ldc = n;
    d.sweep = true; d.sw_k0 = k0; d.sw_kn = kn; d.R = R; d.ldr = n;
    e = gemm(P64, d, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
__global__ void conj_transpose_kernel(int n, const z64* a, z64* at) {
  __shared__ z64 t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 256 threads: 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    if (i < n && j < n) t[r][tx] = a[(long)i * n + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bx + r, j = by + tx;  // at[i][j] = conj(a[j][i])
    if (i < n && j < n) at[(long)i * n + j] = cconj(t[tx][r]);
  }
}

hipError_t conj_transpose(int n, const void* a, void* at, hipStream_t st) {
  hipLaunchKernelGGL(conj_transpose_kernel, dim3(cdiv(n, 32), cdiv(n, 32)), dim3(256), 0, st, n,
                     (const z64*)a, (z64*)at);
  return hipGetLastError();
}

template <typename S, typename D>
__global__ void convert_kernel(const S* src, D* dst, long count2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count2) dst[i] = (D)src[i];
}

hipError_t convert_z(const void* src, bool src32, void* dst, bool dst32, long count, hipStream_t st) {
  const long c2 = 2 * count;
  const unsigned grid = cdiv(c2, 256);
  if (count == 0) return hipSuccess;
  if (src32 && dst32) hipLaunchKernelGGL((convert_kernel<float, float>), dim3(grid), dim3(256), 0, st, (const float*)src, (float*)dst, c2);
  else if (src32) hipLaunchKernelGGL((convert_kernel<float, double>), dim3(grid), dim3(256), 0, st, (const float*)src, (double*)dst, c2);
  else if (dst32) hipLaunchKernelGGL((convert_kernel<double, float>), dim3(grid), dim3(256), 0, st, (const double*)src, (float*)dst, c2);
  else hipLaunchKernelGGL((convert_kernel<double, double>), dim3(grid), dim3(256), 0, st, (const double*)src, (double*)dst, c2);
  return hipGetLastError();
}

__global__ void scale_kernel(const double* src, double* dst, long count2, double alpha) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count2) dst[i] = alpha * src[i];
}

hipError_t scale_z(const void* src, void* dst, long count, double alpha, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_kernel, dim3(cdiv(2 * count, 256)), dim3(256), 0, st, (const double*)src,
                     (double*)dst, 2 * count, alpha);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void frob_partial_kernel(const double* a, long count2, double* partial) {
  __shared__ double red[256];
  double s = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count2; i += (long)gridDim.x * 256) s += a[i] * a[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void sum_kernel(const double* partial, int np, double* out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t frob2(const void* a, long count, double* partial, double* out, hipStream_t st) {
  const long c2 = 2 * count;
  int nb = (int)cdiv(c2, 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(frob_partial_kernel, dim3(nb), dim3(256), 0, st, (const double*)a, c2, partial);
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, (const double*)partial, nb, out);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void diag_min_kernel(const z64* a, int n, double* out) {
  __shared__ double red[256];
  double m = 1e300;
  for (int i = threadIdx.x; i < n; i += 256) m = fmin(m, a[(long)i * n + i].re);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t diag_min(const void* a, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(diag_min_kernel, dim3(1), dim3(256), 0, st, (const z64*)a, n, out);
  return hipGetLastError();
}

}  // namespace isdf
