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
#include "kmajor.h"

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

// ---------------------------------------------------------------------------
// The y and x stages of the adjoint DFT on FP64 MFMA, for lists with at most 32 x- and
// y-frequencies and slabs of at most 64 x 64.  A workgroup of four waves walks an equal
// run of (point, z-plane) slabs.  Per slab:
//   y stage  T1 (y x a)   = CY (y x b) . T2F (b x a)
//   x stage  slab (y x x) = T1 (y x a) . CX (a x x)
// CY[y][b] = conj(twy[b][y]) and CX[a][x] = conj(twx[a][x]) stay in LDS for the whole
// run; T2F is the slab's t2b values of the listed (a, b) pairs placed in a dense block
// whose other entries are zero (set once: the pair set is the same on every slab).
// Padding rows and columns of CY, CX are zero, so padded terms add exactly zero.  The
// slab goes straight from the accumulators to gz.  Two barriers per slab: after the
// T2F scatter (every wave is past the previous slab's x stage, so T1 is free), and
// after T1 is written (every wave is past this slab's y stage, so T2F is free).
// ---------------------------------------------------------------------------
constexpr int AXY_NT = 256;
constexpr int AXY_LD = 65;    // row stride (complex) of the y- and x-indexed arrays
constexpr int AXY_LDA = 33;   // row stride of T2F (a-indexed)
constexpr int AXY_KMAX = 32;  // x- and y-frequencies held
constexpr int AXY_PF = 4;     // pairs per thread (nd <= kx ky <= 1024)

size_t axy_lds_bytes(int kxp, int kyp) {
  return sizeof(z64) * ((size_t)kyp * AXY_LD + (size_t)kyp * AXY_LDA + 2 * (size_t)kxp * AXY_LD);
}

// One 16-deep k block of the wave's FM x FN MFMAs: C += A B with A read k-major
// (As[k][m], stride lda) and B k-major (Bs[k][n], stride ldb), complex128 on the
// real block form (see tile.h).  Fragments with no live row or column are skipped
// (wave-uniform).
template <int FM, int FN>
__device__ __forceinline__ void axy_step(const z64* __restrict__ As, int lda, const z64* __restrict__ Bs, int ldb,
                                         d4 (&acc)[FM][FN], int wm0, int wn0, int mlim, int nlim, int lane) {
  const double* Ar = reinterpret_cast<const double*>(As);
  const double* Br = reinterpret_cast<const double*>(Bs);
  const int i = lane & 15, q = lane >> 4;
  const int bpart = ((q & 1) == (i & 1)) ? 0 : 1;
  const double bsign = ((q & 1) == 1 && (i & 1) == 0) ? -1.0 : 1.0;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    const int k = 2 * kk + (q >> 1);
    double a[FM], b[FN];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm) a[fm] = Ar[(k * lda + wm0 + fm * 16 + i) * 2 + (q & 1)];
#pragma unroll
    for (int fn = 0; fn < FN; ++fn) b[fn] = bsign * Br[(k * ldb + wn0 + fn * 8 + (i >> 1)) * 2 + bpart];
#pragma unroll
    for (int fm = 0; fm < FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < FN; ++fn)
        if (wm0 + fm * 16 < mlim && wn0 + fn * 8 < nlim)
          acc[fm][fn] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[fm], b[fn], acc[fm][fn], 0, 0, 0);
  }
}

__global__ __launch_bounds__(AXY_NT) void adj_xy_kernel(AdjDft p, int kxp, int kyp, long nslab_total, int g,
                                                        const z64* __restrict__ t2b, z64* __restrict__ gz) {
  extern __shared__ unsigned char lds_raw[];
  z64* cy = reinterpret_cast<z64*>(lds_raw);   // [b][y]
  z64* t2f = cy + kyp * AXY_LD;                // [b][a]
  z64* t1 = t2f + kyp * AXY_LDA;               // [a][y]
  z64* cxs = t1 + kxp * AXY_LD;                // [a][x]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const z64* twx = reinterpret_cast<const z64*>(p.twx);
  const z64* twy = reinterpret_cast<const z64*>(p.twy);
  for (int i = tid; i < kyp * AXY_LD; i += AXY_NT) {
    const int b = i / AXY_LD, y = i % AXY_LD;
    const bool ok = b < p.ky && y < p.n1;
    const z64 v = twy[ok ? (long)b * p.n1 + y : 0];
    cy[i] = z64{ok ? v.re : 0.0, ok ? -v.im : 0.0};
  }
  for (int i = tid; i < kxp * AXY_LD; i += AXY_NT) {
    const int a = i / AXY_LD, x = i % AXY_LD;
    const bool ok = a < p.kx && x < p.n0;
    const z64 v = twx[ok ? (long)a * p.n0 + x : 0];
    cxs[i] = z64{ok ? v.re : 0.0, ok ? -v.im : 0.0};
    t1[i] = z64{0.0, 0.0};
  }
  for (int i = tid; i < kyp * AXY_LDA; i += AXY_NT) t2f[i] = z64{0.0, 0.0};
  // this thread's pairs: LDS offset in T2F, or -1
  int off[AXY_PF];
#pragma unroll
  for (int e = 0; e < AXY_PF; ++e) {
    const int d = tid + e * AXY_NT;
    off[e] = d < p.nd ? p.d_by[d] * AXY_LDA + p.d_ax[d] : -1;
  }
  const long s0 = nslab_total * blockIdx.x / g, s1 = nslab_total * (blockIdx.x + 1) / g;
  const int nd = p.nd, n2 = p.n2;
  // t2b offsets of this thread's pairs on slab s: (mu nd + d) n2 + z
  long src[AXY_PF];
#pragma unroll
  for (int e = 0; e < AXY_PF; ++e) src[e] = tid + e * AXY_NT < nd ? (long)(tid + e * AXY_NT) * n2 : -1;
  double pvr[AXY_PF], pvi[AXY_PF];   // split re / im keeps the prefetch in registers
  if (s0 < s1) {
    const long base = (s0 / n2) * nd * n2 + s0 % n2;
#pragma unroll
    for (int e = 0; e < AXY_PF; ++e) {
      const z64 v = t2b[src[e] >= 0 ? base + src[e] : 0];
      pvr[e] = v.re; pvi[e] = v.im;
    }
  }
  const int rc = lane & 15, part = rc & 1;
  const int wm0 = (wave & 1) * 32;
  const int yn0 = (wave >> 1) * 16, xn0 = (wave >> 1) * 32;
  const int n1p = (p.n1 + 15) & ~15;
  const long nslab = (long)p.n0 * p.n1;
  double* t1r = reinterpret_cast<double*>(t1);
  double* gzr = reinterpret_cast<double*>(gz);
  for (long s = s0; s < s1; ++s) {
    if (s == s0) __syncthreads();   // the tables and zeros are in place
#pragma unroll
    for (int e = 0; e < AXY_PF; ++e)
      if (off[e] >= 0) t2f[off[e]] = z64{pvr[e], pvi[e]};
    if (s + 1 < s1) {   // the next slab's pairs, under this slab's MFMAs
      const long base = ((s + 1) / n2) * nd * n2 + (s + 1) % n2;
#pragma unroll
      for (int e = 0; e < AXY_PF; ++e) {
        const z64 v = t2b[src[e] >= 0 ? base + src[e] : 0];
        pvr[e] = v.re; pvi[e] = v.im;
      }
    }
    __syncthreads();
    d4 acc1[2][2];
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
      for (int fn = 0; fn < 2; ++fn) acc1[fm][fn] = d4{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < kyp; kc += 16)
      axy_step<2, 2>(cy + kc * AXY_LD, AXY_LD, t2f + kc * AXY_LDA, AXY_LDA, acc1, wm0, yn0, n1p, kxp, lane);
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
      for (int fn = 0; fn < 2; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int y = wm0 + fm * 16 + Mfma<double>::row(lane, v);
          const int a = yn0 + fn * 8 + (rc >> 1);
          if (a < kxp) t1r[(a * AXY_LD + y) * 2 + part] = acc1[fm][fn][v];
        }
    __syncthreads();
    d4 acc2[2][4];
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn) acc2[fm][fn] = d4{0.0, 0.0, 0.0, 0.0};
    for (int kc = 0; kc < kxp; kc += 16)
      axy_step<2, 4>(t1 + kc * AXY_LD, AXY_LD, cxs + kc * AXY_LD, AXY_LD, acc2, wm0, xn0, n1p, p.n0, lane);
    const int mu = (int)(s / p.n2), z = (int)(s % p.n2);
    double* dst = gzr + ((long)mu * p.n2 + z) * nslab * 2;
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
      for (int fn = 0; fn < 4; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int y = wm0 + fm * 16 + Mfma<double>::row(lane, v);
          const int x = xn0 + fn * 8 + (rc >> 1);
          if (y < p.n1 && x < p.n0) dst[((long)y * p.n0 + x) * 2 + part] = acc2[fm][fn][v];
        }
  }
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
  if (a.kx <= AXY_KMAX && a.ky <= AXY_KMAX && a.n0 <= 64 && a.n1 <= 64 && a.nd <= AXY_PF * AXY_NT) {
    const int kxp = (a.kx + 15) & ~15, kyp = (a.ky + 15) & ~15;
    const size_t lds = axy_lds_bytes(kxp, kyp);
    static bool attr_set[64] = {};  // once per device, for the largest tables
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev < 0 || dev >= 64 || !attr_set[dev]) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&adj_xy_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)axy_lds_bytes(AXY_KMAX, AXY_KMAX));
      if (dev >= 0 && dev < 64) attr_set[dev] = true;
    }
    const long S = (long)a.nmu * a.n2;
    const int g = (int)std::min<long>(S, cu_count());
    hipLaunchKernelGGL(adj_xy_kernel, dim3(g), dim3(AXY_NT), lds, st, a, kxp, kyp, S, g, (const z64*)t2b, (z64*)gz);
    return hipGetLastError();
  }
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
