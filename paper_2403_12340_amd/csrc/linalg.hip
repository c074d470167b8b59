// FP64 dense algebra on the N_mu x N_mu core (row-major complex128, ld = n).
//
//   sweep_inverse  blocked Gauss-Jordan sweep of a Hermitian positive definite
//                  matrix, A <- -A^{-1}, one kernel per 32-wide pivot block.
// A non-positive or non-finite pivot sets bit 0 of *status (ISDF_E_NOT_PD);
// the pivots of a Hermitian positive definite matrix stay positive throughout.
#include "internal.h"
#include "tile.h"

#include <cmath>

namespace isdf {

constexpr int NB = 32;

// 1 / z via the hardware reciprocal of |z|^2 refined by two Newton steps
// (relative error at the level of a few ulp, ample for pivots of a Hermitian
// positive definite elimination).
__device__ __forceinline__ z64 zrcp(z64 z) {
  const double s = z.re * z.re + z.im * z.im;
  double x = __builtin_amdgcn_rcp(s);
  x = x * (2.0 - s * x);
  x = x * (2.0 - s * x);
  return z64{z.re * x, -z.im * x};
}

__device__ __forceinline__ z64 zdiv(z64 a, z64 b) {
  const double d = b.re * b.re + b.im * b.im;
  return z64{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}

// One pivot step of the sweep as a single kernel.  With pivot rows
// k = [k0, k0 + kn) and P = A_kk^{-1}, the swept matrix is
//   A'_kj = P A_kj (j outside k),  A'_ik = A_ik P = (P A_ki)^H (i outside k),
//   A'_kk = -P,  A'_ij = A_ij - A_ik P A_kj = A_ij - conj(A_ki)^T (P A_kj).
// Every workgroup owns one 64 x 64 output tile: it inverts the pivot block in
// LDS by Gauss-Jordan (no pivoting: Hermitian positive definite), forms the
// slices of R = P A_k: it needs, and applies the rank-kn update with MFMA.
// Input and output are different buffers, so no workgroup reads what another
// one writes.
typedef Tile<double, 64, 64, NB, 2, 2> TS;
typedef Tile<double, NB, 64, NB, 2, 2> TP;   // P (NB x NB, k-major in W) times a NB x 64 panel

__global__ __launch_bounds__(256) void sweep_step_kernel(int n, const z64* __restrict__ ain,
                                                         z64* __restrict__ aout, int k0, int kn,
                                                         int* status, int ntm, int total) {
  __shared__ z64 W[NB][NB + 1];   // P = inverse of the (identity-padded) pivot block
  __shared__ z64 rowb[2][NB], colb[2][NB];
  __shared__ z64 As[TS::AS];   // [t][i] = conj(A[k0 + t][m0 + i])   (A operand, k-major)
  __shared__ z64 Bs[TS::BS];   // [t][j] = (P A_k:)[t][n0 + j]        (B operand, k-major)
  __shared__ z64 Ri[NB][64 + 1];  // (P A_k:)[t][m0 + i], only for tiles meeting the pivot columns
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  const int bm = id % ntm, bn = id / ntm;
  const int m0 = bm * 64, n0 = bn * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool need_ri = (n0 < k0 + kn) && (n0 + 64 > k0);
  const int wm0 = (wave % TS::WGM) * TS::WTM, wn0 = (wave / TS::WGM) * TS::WTN;
  const int rc = lane & 15, part = rc & 1;
  const double* ainr = reinterpret_cast<const double*>(ain);

  // this lane's old tile values, loaded first so their latency hides behind the pivot inversion
  double cold[TS::FM][TS::FN][4];
#pragma unroll
  for (int fm = 0; fm < TS::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TS::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + fm * 16 + Mfma<double>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        const long off = (row < n && col < n) ? ((long)row * n + col) * 2 + part : 0;
        cold[fm][fn][v] = ainr[off];
      }
  // pivot block: thread owns column j = tid % 32 of rows r_e = tid / 32 + 8 e (registers)
  constexpr int EW = NB * NB / 256;
  const int gj = tid % NB, gr = tid / NB;
  z64 w[EW];
#pragma unroll
  for (int e = 0; e < EW; ++e) {
    const int r = gr + 8 * e;
    w[e] = (r < kn && gj < kn) ? ain[(long)(k0 + r) * n + k0 + gj] : z64{r == gj ? 1.0 : 0.0, 0.0};
  }
  // raw pivot rows at this tile's columns (into Bs) and rows (into As, conjugated later)
#pragma unroll
  for (int e = 0; e < NB * 64 / 256; ++e) {
    const int idx = tid + 256 * e, t = idx >> 6, c = idx & 63;
    z64 vj{0.0, 0.0}, vi{0.0, 0.0};
    if (t < kn) {
      if (n0 + c < n) vj = ain[(long)(k0 + t) * n + n0 + c];
      if (m0 + c < n) vi = ain[(long)(k0 + t) * n + m0 + c];
    }
    Bs[t * TS::LDB + c] = vj;
    As[t * TS::LDA + c] = vi;
  }
  // Gauss-Jordan in registers: per pivot, the owners publish row p and column p
  // (double-buffered), one barrier, then every thread updates its own elements.
  bool bad_any = false;
#pragma unroll 1
  for (int p = 0; p < NB; ++p) {
    const int b = p & 1;
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      if (gr + 8 * e == p) rowb[b][gj] = w[e];
      if (gj == p) colb[b][gr + 8 * e] = w[e];
    }
    __syncthreads();
    const z64 piv = rowb[b][p];
    const bool bad = !(piv.re > 0.0) || !isfinite(piv.re) || !isfinite(piv.im);
    bad_any |= bad;
    const z64 d = bad ? z64{1.0, 0.0} : zrcp(piv);
    const z64 rv = rowb[b][gj];
    const z64 rs = cmul(rv, d);
    const z64 rj = (gj == p) ? d : rs;   // scaled pivot row at this thread's column
    z64 cv[EW];
#pragma unroll
    for (int e = 0; e < EW; ++e) cv[e] = colb[b][gr + 8 * e];
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const z64 x = cmul(cv[e], rj);
      const double br = (gj == p) ? 0.0 : w[e].re, bi = (gj == p) ? 0.0 : w[e].im;
      const bool own = (gr + 8 * e == p);
      w[e] = z64{own ? rj.re : br - x.re, own ? rj.im : bi - x.im};
    }
  }
  if (bad_any && tid == 0 && id == 0) atomicOr(status, 1);
  // P stored transposed, W[u][t] = P[t][u]: the k-major A operand of P (.) below
#pragma unroll
  for (int e = 0; e < EW; ++e) W[gj][gr + 8 * e] = w[e];
  __syncthreads();
  // Row-panel slices with MFMA: Rj = P A_k(:, tile columns), Ri = P A_k(:, tile rows)
  {
    const int pm0 = (wave % TP::WGM) * TP::WTM, pn0 = (wave / TP::WGM) * TP::WTN;
    TP::acc_t rj[TP::FM][TP::FN], ri[TP::FM][TP::FN];
    zero_acc<TP>(rj);
    tile_mma<double, TP>(&W[0][0], Bs, rj, pm0, pn0, lane);
    if (need_ri) {
      zero_acc<TP>(ri);
      tile_mma<double, TP>(&W[0][0], As, ri, pm0, pn0, lane);
    }
    __syncthreads();  // every wave is done reading the raw panels
    double* Bsr = reinterpret_cast<double*>(Bs);
    double* Rir = reinterpret_cast<double*>(&Ri[0][0]);
#pragma unroll
    for (int fn = 0; fn < TP::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = pm0 + Mfma<double>::row(lane, v);
        const int c = pn0 + fn * 8 + (rc >> 1);
        const int gjc = n0 + c, gic = m0 + c;
        // pivot columns take -P
        const z64 pj = W[(gjc - k0) & (NB - 1)][t];
        const z64 pi = W[(gic - k0) & (NB - 1)][t];
        const bool jp = gjc >= k0 && gjc < k0 + kn, ip = gic >= k0 && gic < k0 + kn;
        Bsr[(t * TS::LDB + c) * 2 + part] = jp ? -(part ? pj.im : pj.re) : rj[0][fn][v];
        if (need_ri) Rir[(t * (64 + 1) + c) * 2 + part] = ip ? -(part ? pi.im : pi.re) : ri[0][fn][v];
      }
    // conjugate the raw pivot rows at this tile's rows into the A operand of the update
#pragma unroll
    for (int e = 0; e < NB * 64 / 256; ++e) {
      const int idx = tid + 256 * e, t = idx >> 6, c = idx & 63;
      As[t * TS::LDA + c].im = -As[t * TS::LDA + c].im;
    }
  }
  __syncthreads();
  TS::acc_t acc[TS::FM][TS::FN];
  zero_acc<TS>(acc);
  tile_mma<double, TS>(As, Bs, acc, wm0, wn0, lane);
  double* aoutr = reinterpret_cast<double*>(aout);
#pragma unroll
  for (int fm = 0; fm < TS::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TS::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + fm * 16 + Mfma<double>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        if (row >= n || col >= n) continue;
        const long off = ((long)row * n + col) * 2 + part;
        double val;
        if (row >= k0 && row < k0 + kn) {
          const z64 r = Bs[(row - k0) * TS::LDB + (col - n0)];
          val = part ? r.im : r.re;
        } else if (col >= k0 && col < k0 + kn) {
          const z64 r = Ri[col - k0][row - m0];
          val = part ? -r.im : r.re;
        } else {
          val = cold[fm][fn][v] - acc[fm][fn][v];
        }
        aoutr[off] = val;
      }
}

size_t linalg_scratch_bytes(int n) { return (size_t)n * n * sizeof(z64); }

hipError_t sweep_inverse(int n, void* a, void* scratch, int* status, hipStream_t st) {
  z64* bufs[2] = {(z64*)a, (z64*)scratch};
  const int ntm = (n + 63) / 64;
  const int total = ntm * ntm;
  const unsigned grid = 8u * (unsigned)((total + 7) / 8);
  int cur = 0;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kn = min(NB, n - k0);
    hipLaunchKernelGGL(sweep_step_kernel, dim3(grid), dim3(256), 0, st, n, (const z64*)bufs[cur],
                       bufs[cur ^ 1], k0, kn, status, ntm, total);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  if (cur == 1) return convert_z(scratch, false, a, false, (long)n * n, st);
  return hipSuccess;
}

// C = a * A + b * B elementwise (complex128, count elements)
__global__ void axpby_kernel(const double* A, double a, const double* B, double b, double* C, long count2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count2) C[i] = a * A[i] + b * B[i];
}

hipError_t axpby(const void* A, double a, const void* B, double b, void* C, long count, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(axpby_kernel, dim3(cdiv(2 * count, 256)), dim3(256), 0, st, (const double*)A, a,
                     (const double*)B, b, (double*)C, 2 * count);
  return hipGetLastError();
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
