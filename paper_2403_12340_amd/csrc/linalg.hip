// FP64 dense algebra on the N_mu x N_mu core (row-major complex128, ld = n).
//
//   sweep_inverse  blocked Gauss-Jordan sweep of a Hermitian positive definite
//                  matrix, A <- -A^{-1}, two kernels per 32-wide pivot block.
// A non-positive or non-finite pivot sets bit 0 of *status (ISDF_E_NOT_PD);
// the pivots of a Hermitian positive definite matrix stay positive throughout.
#include "internal.h"
#include "tile.h"

#include <cmath>

namespace isdf {

constexpr int NB = 32;

// 1 / x for a positive pivot: hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double drcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  r = r * (2.0 - x * r);
  return r;
}

// One 32-pivot step of the sweep is two kernels.  With pivot rows
// k = [k0, k0 + kn), P = A_kk^{-1} and R = P A_k: (kn x n),
//   A'_kj = R_j (j outside k),  A'_kk = -P,
//   A'_ik = A_ik P = (P A_ki)^H = R_i^H (i outside k; A stays Hermitian),
//   A'_ij = A_ij - A_ik P A_kj = A_ij - sum_t conj(A[k0 + t][i]) R[t][j].
// sweep_panel_kernel writes the pivot rows and columns of A' (one workgroup per
// 64-column block), sweep_update_kernel the rest.  Input and output are
// different buffers, so no workgroup reads what another one writes.
//
// The pivot block is inverted by in-register Gauss-Jordan.  After pivots
// 0..p-1 the working block B satisfies B[r][j] = s conj(B[j][r]) with s = -1
// exactly when one of r, j is already a pivot, so row p alone carries what
// every thread needs: the column value is B[r][p] = s conj(B[p][r]).  One row
// broadcast and one barrier per pivot.
typedef Tile<double, NB, 64, NB, 2, 2> TP;   // P (NB x NB, k-major in W) times a NB x 64 panel

// Gauss-Jordan inversion of the NB x NB pivot block held as w[e] = B[gr + 8 e][gj]
// by 256 threads (identity padding beyond the block); returns whether a pivot was
// not positive and finite.  One row broadcast through rowb and one barrier per pivot.
constexpr int EW = NB * NB / 256;
__device__ __forceinline__ bool pivot_gj(z64 (&w)[EW], z64 (*rowb)[NB], int gj, int gr) {
  bool bad_any = false;
#pragma unroll
  for (int p = 0; p < NB; ++p) {
    const int b = p & 1;
    if (gr == (p & 7)) rowb[b][gj] = w[p >> 3];
    __syncthreads();
    const double piv = rowb[b][p].re;
    const bool bad = !(piv > 0.0) || !isfinite(piv);
    bad_any |= bad;
    const double d = bad ? 1.0 : drcp(piv);
    const z64 rv = rowb[b][gj];
    const z64 rj = (gj == p) ? z64{d, 0.0} : z64{rv.re * d, rv.im * d};  // scaled pivot row here
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int r = gr + 8 * e;
      const z64 pr = rowb[b][r];                 // B[p][r]
      const double sg = (r < p) ? -1.0 : 1.0;    // B[r][p] = sg conj(B[p][r])
      const z64 cv{sg * pr.re, -sg * pr.im};
      const z64 x = cmul(cv, rj);
      const double br = (gj == p) ? 0.0 : w[e].re, bi = (gj == p) ? 0.0 : w[e].im;
      const bool own = (r == p);
      w[e] = z64{own ? rj.re : br - x.re, own ? rj.im : bi - x.im};
    }
  }
  return bad_any;
}

// pin: P of this step (W layout, P[t][u] at pin[u NB + t]) when the previous
// update launch computed it, else null (the panel inverts the block itself)
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void sweep_panel_kernel(int n, const z64* __restrict__ ain,
                                                          z64* __restrict__ aout, int k0, int kn,
                                                          const z64* __restrict__ pin, int* status) {
  // The sweep steps are latency-bound and run beside the pair kernel's waves: their
  // waves take issue priority on the SIMDs they share.
  __builtin_amdgcn_s_setprio(3);
  ain += (long)blockIdx.y * n * n;   // batch item
  aout += (long)blockIdx.y * n * n;
  __shared__ z64 W[NB][NB + 1];      // W[u][t] = P[t][u]: the k-major A operand of P (.)
  __shared__ z64 rowb[2][NB];        // pivot row broadcast, double-buffered
  __shared__ z64 Bs[NB * (64 + 1)];  // pivot rows at this block's columns, then R
  const int c0 = blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // pivot block first: Gauss-Jordan waits only for these loads.
  // Thread owns column gj of rows gr + 8 e (identity padding beyond kn).
  const int gj = tid % NB, gr = tid / NB;
  if (pin) pin += (long)blockIdx.y * NB * NB;
  z64 w[EW];
  if (!pin) {
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int r = gr + 8 * e;
      const bool ok = r < kn && gj < kn;
      const z64 v = ain[ok ? (long)(k0 + r) * n + k0 + gj : 0];
      w[e] = ok ? v : z64{r == gj ? 1.0 : 0.0, 0.0};
    }
  }
  // raw pivot rows at this block's columns, kept in registers until the inversion is done
  constexpr int EB = NB * 64 / 256;
  z64 braw[EB];
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    const int idx = tid + 256 * e, t = idx >> 6, c = idx & 63;
    const bool ok = t < kn && c0 + c < n;
    braw[e] = ain[ok ? (long)(k0 + t) * n + c0 + c : 0];
  }
  bool bad_any = false;
  if (pin) {
    // P precomputed by the previous step's update launch
#pragma unroll
    for (int e = 0; e < EW; ++e) w[e] = pin[gj * NB + gr + 8 * e];
  } else {
    bad_any = pivot_gj(w, rowb, gj, gr);
  }
  if (bad_any && tid == 0 && blockIdx.x == 0) atomicOr(status, 1);
#pragma unroll
  for (int e = 0; e < EW; ++e) W[gj][gr + 8 * e] = w[e];
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    const int idx = tid + 256 * e, t = idx >> 6, c = idx & 63;
    const bool ok = t < kn && c0 + c < n;
    Bs[t * (64 + 1) + c] = ok ? braw[e] : z64{0.0, 0.0};
  }
  __syncthreads();
  // R = P A_k(:, block columns) with MFMA
  const int pm0 = (wave % TP::WGM) * TP::WTM, pn0 = (wave / TP::WGM) * TP::WTN;
  const int rc = lane & 15, part = rc & 1;
  TP::acc_t racc[TP::FM][TP::FN];
  zero_acc<TP>(racc);
  tile_mma<double, TP>(&W[0][0], Bs, racc, pm0, pn0, lane);
  __syncthreads();  // every wave is done reading the raw panel
  double* Bsr = reinterpret_cast<double*>(Bs);
#pragma unroll
  for (int fn = 0; fn < TP::FN; ++fn)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int t = pm0 + Mfma<double>::row(lane, v);
      const int c = pn0 + fn * 8 + (rc >> 1);
      const int gc = c0 + c;
      const bool piv_col = gc >= k0 && gc < k0 + kn;
      const z64 pv = W[(gc - k0) & (NB - 1)][t];  // P[t][gc - k0]
      Bsr[(t * (64 + 1) + c) * 2 + part] = piv_col ? -(part ? pv.im : pv.re) : racc[0][fn][v];
    }
  __syncthreads();
  // pivot rows: A'[k0 + t][c0 + c] (coalesced along c)
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    const int idx = tid + 256 * e, t = idx >> 6, c = idx & 63;
    if (t < kn && c0 + c < n) aout[(long)(k0 + t) * n + c0 + c] = Bs[t * (64 + 1) + c];
  }
  // pivot columns: A'[i][k0 + t] = conj(R[t][i]) for rows i of this block outside k (coalesced along t)
#pragma unroll
  for (int e = 0; e < EB; ++e) {
    const int idx = tid + 256 * e, t = idx & (NB - 1), c = idx / NB;
    const int i = c0 + c;
    if (t < kn && i < n && !(i >= k0 && i < k0 + kn)) aout[(long)i * n + k0 + t] = cconj(Bs[t * (64 + 1) + c]);
  }
}

// Rank-kn update of every element outside the pivot rows and columns.
typedef Tile<double, 64, 32, 16, 2, 2> TU;

// With pout set, one more workgroup (the last) looks ahead: it forms the next
// pivot block k1 of A' (kn1 wide) from the same formula, inverts it by
// Gauss-Jordan while the others update, and stores P for the next panel launch,
// so that the serial inversion is off the critical path of every step but the first.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void sweep_update_kernel(int n, const z64* __restrict__ ain,
                                                           z64* __restrict__ aout, int k0, int kn,
                                                           int ntm, int total, z64* __restrict__ pout,
                                                           int k1, int kn1, int* status) {
  __shared__ z64 As[TU::AS];  // [t][i] = conj(A[k0 + t][m0 + i])
  __shared__ z64 Bs[TU::BS];  // [t][j] = R[t][n0 + j] (the pivot rows of A')
  __builtin_amdgcn_s_setprio(3);   // issue priority beside the pair kernel, as in the panel
  ain += (long)blockIdx.y * n * n;   // batch item
  aout += (long)blockIdx.y * n * n;
  if (pout && blockIdx.x == gridDim.x - 1) {
    pout += (long)blockIdx.y * NB * NB;
    const int tid = threadIdx.x, gj = tid % NB, gr = tid / NB;
    const bool colok = gj < kn1;
    // sum_t conj(A[k0 + t][k1 + r]) R[t][k1 + gj], t in halves of 16 staged in LDS:
    // As[t][r] = A[k0 + t][k1 + r], Bs[t][u] = R[t][k1 + u] (stride 33; zero beyond the blocks)
    static_assert(TU::AS >= 16 * 33 && TU::BS >= 16 * 33, "look-ahead staging fits the tile buffers");
    z64 vold[EW];
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int r = gr + 8 * e;
      vold[e] = ain[r < kn1 && colok ? (long)(k1 + r) * n + k1 + gj : 0];
    }
    z64 acc[EW];
#pragma unroll
    for (int e = 0; e < EW; ++e) acc[e] = z64{0.0, 0.0};
    for (int t0 = 0; t0 < kn; t0 += 16) {
      z64 sa[2], sb[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {   // element (t, c) = (idx / 32, idx % 32), idx = tid + 256 h
        const int idx = tid + 256 * h, t = idx >> 5, c = idx & 31;
        const bool tok = t0 + t < kn && c < kn1;
        sa[h] = ain[tok ? (long)(k0 + t0 + t) * n + k1 + c : 0];
        sb[h] = aout[tok ? (long)(k0 + t0 + t) * n + k1 + c : 0];
        if (!tok) sa[h] = sb[h] = z64{0.0, 0.0};
      }
      __syncthreads();   // the previous half has been read
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int idx = tid + 256 * h, t = idx >> 5, c = idx & 31;
        As[t * 33 + c] = sa[h];
        Bs[t * 33 + c] = sb[h];
      }
      __syncthreads();
#pragma unroll 4
      for (int t = 0; t < 16; ++t) {
        const z64 rv = Bs[t * 33 + gj];
#pragma unroll
        for (int e = 0; e < EW; ++e) {
          const z64 x = cmulc(As[t * 33 + gr + 8 * e], rv);
          acc[e].re += x.re;
          acc[e].im += x.im;
        }
      }
    }
    __syncthreads();   // As is reused as the pivot-row broadcast
    z64 w[EW];
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int r = gr + 8 * e;
      const bool ok = r < kn1 && colok;
      w[e] = ok ? z64{vold[e].re - acc[e].re, vold[e].im - acc[e].im} : z64{r == gj ? 1.0 : 0.0, 0.0};
    }
    z64 (*rowb)[NB] = reinterpret_cast<z64 (*)[NB]>(As);
    const bool bad = pivot_gj(w, rowb, gj, gr);
    if (bad && tid == 0) atomicOr(status, 1);
#pragma unroll
    for (int e = 0; e < EW; ++e) pout[gj * NB + gr + 8 * e] = w[e];
    return;
  }
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  const int bm = id % ntm, bn = id / ntm;
  const int m0 = bm * TU::BM, n0 = bn * TU::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % TU::WGM) * TU::WTM, wn0 = (wave / TU::WGM) * TU::WTN;
  const int rc = lane & 15, part = rc & 1;
  Stager<double, double, TU::BM, TU::BK, TU::NT, true> sa;
  Stager<double, double, TU::BN, TU::BK, TU::NT, true> sb;
  sa.fetch(ain + (long)k0 * n, 1, n, m0, 0, n, kn, tid);
  sb.fetch(aout + (long)k0 * n, 1, n, n0, 0, n, kn, tid);
  const double* ainr = reinterpret_cast<const double*>(ain);
  double cold[TU::FM][TU::FN][4];
#pragma unroll
  for (int fm = 0; fm < TU::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TU::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + fm * 16 + Mfma<double>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        // 32-bit byte offsets from the uniform base: one address register per load
        const unsigned off = (row < n && col < n) ? ((unsigned)(row * n + col) * 2u + part) * 8u : 0u;
        cold[fm][fn][v] = *reinterpret_cast<const double*>(reinterpret_cast<const char*>(ainr) + off);
      }
  TU::acc_t acc[TU::FM][TU::FN];
  zero_acc<TU>(acc);
  for (int kc = 0; kc < kn; kc += TU::BK) {
    sa.store(As, TU::LDA, -1.0, tid);
    sb.store(Bs, TU::LDB, 1.0, tid);
    __syncthreads();
    if (kc + TU::BK < kn) {
      sa.fetch(ain + (long)k0 * n, 1, n, m0, kc + TU::BK, n, kn, tid);
      sb.fetch(aout + (long)k0 * n, 1, n, n0, kc + TU::BK, n, kn, tid);
    }
    tile_mma<double, TU>(As, Bs, acc, wm0, wn0, lane);
    __syncthreads();
  }
  double* aoutr = reinterpret_cast<double*>(aout);
#pragma unroll
  for (int fm = 0; fm < TU::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TU::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + fm * 16 + Mfma<double>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        if (row >= n || col >= n) continue;
        if ((row >= k0 && row < k0 + kn) || (col >= k0 && col < k0 + kn)) continue;
        aoutr[((long)row * n + col) * 2 + part] = cold[fm][fn][v] - acc[fm][fn][v];
      }
}

// ping-pong copy of the matrix, then the look-ahead pivot inverse
size_t linalg_scratch_bytes(int n) { return ((size_t)n * n + NB * NB) * sizeof(z64); }

hipError_t sweep_inverse(int n, void* a, void* scratch, int* status, hipStream_t st, int batch) {
  z64* bufs[2] = {(z64*)a, (z64*)scratch};
  const int npb = (n + 63) / 64;                  // panel workgroups
  const int ntm = (n + TU::BM - 1) / TU::BM, ntn = (n + TU::BN - 1) / TU::BN;
  const int total = ntm * ntn;
  const unsigned grid = 8u * (unsigned)((total + 7) / 8);
  z64* pbuf = (z64*)scratch + (long)batch * n * n;   // look-ahead P, one block per batch item
  int cur = 0;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kn = min(NB, n - k0);
    hipLaunchKernelGGL(sweep_panel_kernel, dim3(npb, batch), dim3(256), 0, st, n, (const z64*)bufs[cur],
                       bufs[cur ^ 1], k0, kn, k0 > 0 ? (const z64*)pbuf : nullptr, status);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int k1 = k0 + NB, kn1 = min(NB, n - k1);
    const bool ahead = k1 < n;
    hipLaunchKernelGGL(sweep_update_kernel, dim3(grid + (ahead ? 1 : 0), batch), dim3(256), 0, st, n,
                       (const z64*)bufs[cur], bufs[cur ^ 1], k0, kn, ntm, total, ahead ? pbuf : nullptr, k1, kn1,
                       status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
  }
  if (cur == 1) return convert_z(scratch, false, a, false, (long)n * n * batch, st);
  return hipSuccess;
}

// Zero `bytes` bytes (a multiple of 4) with a kernel, so that the clear can sit in
// a captured graph.
__global__ void zero_kernel(uint32_t* p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

hipError_t zero_fill(void* p, size_t bytes, hipStream_t st) {
  const long n = (long)(bytes / 4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(zero_kernel, dim3(cdiv(n, 256)), dim3(256), 0, st, (uint32_t*)p, n);
  return hipGetLastError();
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

// smallest real diagonal entry over `batch` n x n matrices stored back to back
__global__ __launch_bounds__(256) void diag_min_kernel(const z64* a, int n, int batch, double* out) {
  __shared__ double red[256];
  double m = 1e300;
  const long nd = (long)n * batch;
  for (long i = threadIdx.x; i < nd; i += 256) {
    const long b = i / n, r = i % n;
    m = fmin(m, a[b * n * n + r * n + r].re);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmin(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

hipError_t diag_min(const void* a, int n, double* out, hipStream_t st, int batch) {
  hipLaunchKernelGGL(diag_min_kernel, dim3(1), dim3(256), 0, st, (const z64*)a, n, batch, out);
  return hipGetLastError();
}

// H[b] = G - K[b] (complex128 as 2 n2 doubles per item)
__global__ void sub_bcast_kernel(const double* G, const double* K, double* H, long n2x2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n2x2) return;
  const long o = (long)blockIdx.y * n2x2 + i;
  H[o] = G[i] - K[o];
}

hipError_t sub_bcast(const void* G, const void* K, void* H, long n2, int batch, hipStream_t st) {
  hipLaunchKernelGGL(sub_bcast_kernel, dim3(cdiv(2 * n2, 256), batch), dim3(256), 0, st, (const double*)G,
                     (const double*)K, (double*)H, 2 * n2);
  return hipGetLastError();
}

}  // namespace isdf
