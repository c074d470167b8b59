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

// 1 / x for a positive pivot: hardware reciprocal refined by two Newton steps.
__device__ __forceinline__ double drcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = r * (2.0 - x * r);
  r = r * (2.0 - x * r);
  return r;
}

// One 32-pivot step of the sweep is one kernel.  With pivot rows k = [k0, k0 + kn)
// and P = A_kk^{-1}:
//   A'_kk = -P,  A'_kj = (P A_k)_j = R_j (j outside k),
//   A'_ik = A_ik P (i outside k),  A'_ij = A_ij - A_ik R_j,
// with A_ik = conj(A_ki) (A stays Hermitian).  The workgroup of a 64 x 32 tile forms
// the R block of its own columns in LDS (P times the 32 x 32 pivot-row block), so no
// separate panel launch is needed; the tile on the pivot columns multiplies by P
// instead.  Input and output are different buffers, so no workgroup reads what
// another one writes.  P comes from the previous step's last workgroup, which forms
// the next pivot block of A' by the same formula and inverts it while the others
// update (look-ahead); the first step's P comes from sweep_first_kernel.
//
// The pivot block is inverted by Gauss-Jordan, two pivots per barrier.  After the
// pivots before p0 the working block B satisfies B[r][j] = s conj(B[j][r]) with
// s = -1 exactly when one of r, j is already a pivot, so the two pivot rows alone
// carry what every thread needs: the 2 x 2 pivot block D (inverted in closed form),
// the pivot-row values at the thread's columns, and the pivot-column values at its
// rows B[r][p0 + a] = s conj(B[p0 + a][r]).  One round is the rank-2 update
//   B' = B~ - C Y,   C[r][a] = B[r][p0 + a] (pivot rows: C = -I),
//   Y[a][j] = (D^{-1} (B[p0][j], B[p0 + 1][j]))_a (pivot columns: D^{-1}[a][j - p0]),
// where B~ is B with its two pivot rows and columns cleared.  In the real block form
// of the complex product this is exactly one 16x16x4 FP64 MFMA per 16-row tile: the
// four k of the MFMA are (re, im) of the two pivots.
//
// Layout: 4 waves; wave w holds the real columns [16 w, 16 w + 16) of both 16-row
// tiles as MFMA accumulators, acc[t][v] = real entry (16 t + 4 v + l / 16, 16 w + l % 16)
// of lane l (complex column (16 w + l % 16) / 2, re or im by the column's parity).
constexpr int GJ_THREADS = 256;
constexpr int EW = NB * NB / GJ_THREADS;   // complex entries of a 32 x 32 block per thread

// Gauss-Jordan inversion of the NB x NB block in acc (identity padding beyond the
// block); rowd: LDS for the two pivot rows as reals, double buffered.  Returns whether
// a 2 x 2 pivot block was not positive definite (every thread returns the same).
__device__ __forceinline__ bool pivot_gj(d4 (&acc)[2], double (*rowd)[2][2 * NB], int lane, int wave) {
  const int kq = lane >> 4, i16 = lane & 15;
  const int jr = 16 * wave + i16, j = jr >> 1, part = jr & 1;   // this lane's real / complex column
  const int ka = kq >> 1, kp = kq & 1;                           // MFMA k = 2 a + p: pivot a, re / im
  bool bad_any = false;
#pragma unroll
  for (int q = 0; q < NB / 2; ++q) {
    const int p0 = 2 * q, b = q & 1;
    // rows p0, p0 + 1 to LDS: tile p / 16, register (p % 16) / 4, lanes with l / 16 = p % 4
    if (kq == (p0 & 3)) rowd[b][0][jr] = acc[p0 >> 4][(p0 & 15) >> 2];
    if (kq == ((p0 + 1) & 3)) rowd[b][1][jr] = acc[(p0 + 1) >> 4][((p0 + 1) & 15) >> 2];
    __syncthreads();
    const double a = rowd[b][0][2 * p0], d = rowd[b][1][2 * p0 + 2];
    const double cre = rowd[b][0][2 * p0 + 2], cim = rowd[b][0][2 * p0 + 3];
    const double v0r = rowd[b][0][2 * j], v0i = rowd[b][0][2 * j + 1];
    const double v1r = rowd[b][1][2 * j], v1i = rowd[b][1][2 * j + 1];
    double xa[2];   // component kp of B[p0 + ka][r], r = 16 t + l % 16
#pragma unroll
    for (int t = 0; t < 2; ++t) xa[t] = rowd[b][ka][2 * (16 * t + i16) + kp];
    __builtin_amdgcn_sched_barrier(0);   // every read of the round in flight at once
    const double det = a * d - (cre * cre + cim * cim);
    const bool bad = !(a > 0.0) || !(det > 0.0) || !isfinite(det);
    bad_any |= bad;
    const double idet = bad ? 0.0 : drcp(det);
    // row ka of D^{-1} = [d, -c; -conj(c), a] / det
    const double e0r = ka == 0 ? d * idet : -cre * idet, e0i = ka == 0 ? 0.0 : cim * idet;
    const double e1r = ka == 0 ? -cre * idet : a * idet, e1i = ka == 0 ? -cim * idet : 0.0;
    double yr = e0r * v0r - e0i * v0i + e1r * v1r - e1i * v1i;
    double yi = e0r * v0i + e0i * v0r + e1r * v1i + e1i * v1r;
    if (j == p0) { yr = e0r; yi = e0i; }
    if (j == p0 + 1) { yr = e1r; yi = e1i; }
    // B operand: entry (k = 2 ka + kp, real column jr) of the real block form of -Y
    const double bop = part == 0 ? (kp == 0 ? -yr : yi) : (kp == 0 ? -yi : -yr);
    const bool jpiv = j == p0 || j == p0 + 1;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int r = 16 * t + i16;
      const double sg = r < p0 ? -1.0 : 1.0;
      // A operand: component kp of C[r][ka] = sg conj(B[p0 + ka][r]); -I on the pivot rows
      double aop = kp == 0 ? sg * xa[t] : -sg * xa[t];
      if (r == p0 || r == p0 + 1) aop = (r - p0 == ka && kp == 0) ? -1.0 : 0.0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * t + 4 * v + kq;
        if (jpiv || row == p0 || row == p0 + 1) acc[t][v] = 0.0;
      }
      acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(aop, bop, acc[t], 0, 0, 0);
    }
  }
  return bad_any;
}

// P = the inverted block from acc into pout (pout[u NB + t] = P[t][u])
__device__ __forceinline__ void store_p(const d4 (&acc)[2], z64* pout, int lane, int wave) {
  const int kq = lane >> 4, jr = 16 * wave + (lane & 15);
  double* pd = reinterpret_cast<double*>(pout);
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) pd[((jr >> 1) * NB + 16 * t + 4 * v + kq) * 2 + (jr & 1)] = acc[t][v];
}

typedef Tile<double, 32, 32, 32, 2, 2> TR;   // R = P A_kj: 32 x 32 x 32
typedef Tile<double, 64, 32, 32, 2, 2> TU;   // the tile update: 64 x 32, K = the 32 pivots
constexpr int LP = NB + 1;                   // row stride of the 32 x 32 LDS blocks

// P of the first pivot block, per batch item (pout[u NB + t] = P[t][u])
__global__ __launch_bounds__(GJ_THREADS) void sweep_first_kernel(int n, const z64* __restrict__ ain,
                                                                 z64* __restrict__ pout, int kn, int* status) {
  __shared__ double rowd[2][2][2 * NB];
  ain += (long)blockIdx.y * n * n;
  pout += (long)blockIdx.y * NB * NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int kq = lane >> 4, jr = 16 * wave + (lane & 15), j = jr >> 1, part = jr & 1;
  const double* ad = reinterpret_cast<const double*>(ain);
  d4 acc[2];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 16 * t + 4 * v + kq;
      const bool ok = r < kn && j < kn;
      const double x = ad[ok ? ((long)r * n + j) * 2 + part : 0];
      acc[t][v] = ok ? x : (r == j && part == 0 ? 1.0 : 0.0);
    }
  const bool bad = pivot_gj(acc, rowd, lane, wave);
  if (bad && tid == 0) atomicOr(status, 1);
  store_p(acc, pout, lane, wave);
}

// R = P K in LDS: Ps[s][t] = P[t][s] (k-major A operand), Ks[s][j] = A[k0 + s][c0 + j];
// R[t][j] to Rs (stride LP)
__device__ __forceinline__ void form_r(const z64* Ps, const z64* Ks, z64* Rs, int lane, int wave) {
  const int wm0 = (wave % TR::WGM) * TR::WTM, wn0 = (wave / TR::WGM) * TR::WTN;
  const int rc = lane & 15, part = rc & 1;
  TR::acc_t acc[TR::FM][TR::FN];
  zero_acc<TR>(acc);
  tile_mma<double, TR>(Ps, Ks, acc, wm0, wn0, lane);
  double* Rr = reinterpret_cast<double*>(Rs);
#pragma unroll
  for (int fm = 0; fm < TR::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TR::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int t = wm0 + fm * 16 + Mfma<double>::row(lane, v);
        const int j = wn0 + fn * 8 + (rc >> 1);
        Rr[(t * LP + j) * 2 + part] = acc[fm][fn][v];
      }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void sweep_step_kernel(
    int n, const z64* __restrict__ ain, z64* __restrict__ aout, int k0, int kn, const z64* __restrict__ pin,
    z64* __restrict__ pout, int k1, int kn1, int ntm, int total, int* status, int prio) {
  // The sweep steps are latency-bound and run beside the pair kernel's waves: with
  // prio set, their waves take issue priority on the SIMDs they share.
  if (prio) __builtin_amdgcn_s_setprio(3);
  __shared__ z64 L0[2 * NB * LP];   // Ps + Ks, later the update's A operand [t][i] (32 x 65)
  __shared__ z64 Rs[NB * LP];       // R [t][j], or P [t][u] on the pivot columns
  static_assert(TU::AS <= 2 * NB * LP && TU::BS <= NB * LP, "update operands fit the LDS blocks");
  z64* Ps = L0;
  z64* Ks = L0 + NB * LP;
  ain += (long)blockIdx.y * n * n;   // batch item
  aout += (long)blockIdx.y * n * n;
  pin += (long)blockIdx.y * NB * NB;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int rc = lane & 15, part = rc & 1;
  if (pout && blockIdx.x == gridDim.x - 1) {
    // look-ahead: A'_{k1 k1} = A_{k1 k1} - conj(A_{k k1})^T R1, R1 = P A_{k k1}; then its inverse
    pout += (long)blockIdx.y * NB * NB;
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int idx = tid + 256 * e, s2 = idx / NB, t = idx % NB;
      Ps[s2 * LP + t] = pin[idx];                                             // P[t][s2]
      const bool ok = s2 < kn && t < kn1;
      const z64 v = ain[ok ? (long)(k0 + s2) * n + k1 + t : 0];
      Ks[s2 * LP + t] = ok ? v : z64{0.0, 0.0};                               // A[k0 + s2][k1 + t]
    }
    // A_{k1 k1} in the elimination's layout (real entry (16 t + 4 v + l / 16, 16 w + l % 16))
    const int kq = lane >> 4, jr = 16 * wave + (lane & 15), j = jr >> 1, part = jr & 1;
    const double* ad = reinterpret_cast<const double*>(ain);
    d4 acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * t + 4 * v + kq;
        acc[t][v] = ad[r < kn1 && j < kn1 ? ((long)(k1 + r) * n + k1 + j) * 2 + part : 0];
      }
    __syncthreads();
    form_r(Ps, Ks, Rs, lane, wave);
    __syncthreads();
    // conj(A_{k k1})^T as the k-major A operand, in Ps's place
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int idx = tid + 256 * e, s2 = idx / NB, t = idx % NB;
      Ps[s2 * LP + t] = cconj(Ks[s2 * LP + t]);
    }
    __syncthreads();
    // C = conj(A_{k k1})^T R1 into Ks's place (its raw values are no longer needed)
    form_r(Ps, Rs, Ks, lane, wave);
    __syncthreads();
    {
      const double* Kd = reinterpret_cast<const double*>(Ks);
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = 16 * t + 4 * v + kq;
          const bool ok = r < kn1 && j < kn1;
          acc[t][v] = ok ? acc[t][v] - Kd[(r * LP + j) * 2 + part] : (r == j && part == 0 ? 1.0 : 0.0);
        }
    }
    __syncthreads();   // Ks read before the pivot rows reuse Rs
    const bool bad = pivot_gj(acc, reinterpret_cast<double (*)[2][2 * NB]>(Rs), lane, wave);
    if (bad && tid == 0) atomicOr(status, 1);
    store_p(acc, pout, lane, wave);
    return;
  }
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  const int bm = id % ntm, bn = id / ntm;
  const int m0 = bm * TU::BM, n0 = bn * TU::BN;
  const bool pcol = n0 == k0;   // the tile on the pivot columns (k0 is a multiple of 32)
  const int wm0 = (wave % TU::WGM) * TU::WTM, wn0 = (wave / TU::WGM) * TU::WTN;
  // the update's A operand conj(A[k0 + t][m0 + i]), in flight while R is formed
  Stager<double, double, TU::BM, TU::BK, TU::NT, true> sa;
  sa.fetch(ain + (long)k0 * n, 1, n, m0, 0, n, kn, tid);
  if (pcol) {
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int idx = tid + 256 * e, u = idx / NB, t = idx % NB;
      Rs[t * LP + u] = pin[idx];                                              // P[t][u]
    }
  } else {
    Stager<double, double, NB, NB, 256, true> sk;
    sk.fetch(ain + (long)k0 * n, 1, n, n0, 0, n, kn, tid);
#pragma unroll
    for (int e = 0; e < EW; ++e) {
      const int idx = tid + 256 * e, s2 = idx / NB, t = idx % NB;
      Ps[s2 * LP + t] = pin[idx];                                             // P[t][s2]
    }
    sk.store(Ks, LP, 1.0, tid);
    __syncthreads();
    form_r(Ps, Ks, Rs, lane, wave);
  }
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
  __syncthreads();   // Ps / Ks read by form_r before the A operand overwrites them
  sa.store(L0, TU::LDA, -1.0, tid);
  __syncthreads();
  TU::acc_t acc[TU::FM][TU::FN];
  zero_acc<TU>(acc);
  tile_mma<double, TU>(L0, Rs, acc, wm0, wn0, lane);
  const double* Rr = reinterpret_cast<const double*>(Rs);
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
        const bool prow = row >= k0 && row < k0 + kn;
        double val;
        if (pcol) val = prow ? -Rr[((row - k0) * LP + (col - k0)) * 2 + part] : acc[fm][fn][v];   // -P, A_ik P
        else val = prow ? Rr[((row - k0) * LP + (col - n0)) * 2 + part] : cold[fm][fn][v] - acc[fm][fn][v];
        aoutr[((long)row * n + col) * 2 + part] = val;
      }
}

// ping-pong copy of the matrix, then the two look-ahead pivot inverses (by step parity)
size_t linalg_scratch_bytes(int n) { return ((size_t)n * n + 2 * NB * NB) * sizeof(z64); }

hipError_t sweep_inverse(int n, void* a, void* scratch, int* status, hipStream_t st, int batch, bool prio,
                         bool first_done) {
  z64* bufs[2] = {(z64*)a, (z64*)scratch};
  z64* pbuf[2] = {(z64*)scratch + (long)batch * n * n, (z64*)scratch + (long)batch * n * n + (long)batch * NB * NB};
  const int ntm = (n + TU::BM - 1) / TU::BM, ntn = (n + TU::BN - 1) / TU::BN;
  const int total = ntm * ntn;
  const unsigned grid = 8u * (unsigned)((total + 7) / 8);
  hipError_t e = hipSuccess;
  if (!first_done) {
    hipLaunchKernelGGL(sweep_first_kernel, dim3(1, batch), dim3(256), 0, st, n, (const z64*)a, pbuf[0], min(NB, n),
                       status);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int cur = 0, par = 0;
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int kn = min(NB, n - k0);
    const int k1 = k0 + NB, kn1 = min(NB, n - k1);
    const bool ahead = k1 < n;
    hipLaunchKernelGGL(sweep_step_kernel, dim3(grid + (ahead ? 1 : 0), batch), dim3(256), 0, st, n,
                       (const z64*)bufs[cur], bufs[cur ^ 1], k0, kn, (const z64*)pbuf[par],
                       ahead ? pbuf[par ^ 1] : nullptr, k1, kn1, ntm, total, status, prio ? 1 : 0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    cur ^= 1;
    par ^= 1;
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

// per-block partial sums of a[i]^2; with c32, a[i] rounded to FP32 there as well
__global__ __launch_bounds__(256) void frob_partial_kernel(const double* a, long count2, double* partial,
                                                           float* c32) {
  __shared__ double red[256];
  double s = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count2; i += (long)gridDim.x * 256) {
    const double x = a[i];
    s += x * x;
    if (c32) c32[i] = (float)x;
  }
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

hipError_t frob2(const void* a, long count, double* partial, double* out, hipStream_t st, void* copy32) {
  const long c2 = 2 * count;
  int nb = (int)cdiv(c2, 256);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(frob_partial_kernel, dim3(nb), dim3(256), 0, st, (const double*)a, c2, partial,
                     (float*)copy32);
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

// H = G - K (n x n complex128) with the two checks of H made before its inversion,
// in one pass: per-block partial sums of |H|^2 (partial[b]) and minima of its real
// diagonal (partial[FH_MAXB + b]); form_h_finish_kernel combines them in fixed order.
// With pfirst, one more workgroup (the last) forms the first 32 x 32 pivot block of H
// from G and K itself and inverts it, as sweep_first_kernel would after this kernel, into
// pfirst (pfirst[u NB + t] = P[t][u]); sweep_inverse is then called with first_done.
constexpr int FH_MAXB = 512;
__global__ __launch_bounds__(256) void form_h_kernel(const double* G, const double* K, double* H, int n,
                                                     long count2, double* partial, z64* pfirst, int* status) {
  __shared__ double rs[256], rm[256];
  __shared__ double rowd[2][2][2 * NB];
  if (pfirst && blockIdx.x == gridDim.x - 1) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int kq = lane >> 4, jr = 16 * wave + (lane & 15), j = jr >> 1, part = jr & 1;
    const int kn = n < NB ? n : NB;
    d4 acc[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * t + 4 * v + kq;
        const bool ok = r < kn && j < kn;
        const long o = ok ? ((long)r * n + j) * 2 + part : 0;
        const double x = G[o] - K[o];
        acc[t][v] = ok ? x : (r == j && part == 0 ? 1.0 : 0.0);
      }
    const bool bad = pivot_gj(acc, rowd, lane, wave);
    if (bad && tid == 0) atomicOr(status, 1);
    store_p(acc, pfirst, lane, wave);
    return;
  }
  double s = 0.0, m = 1e300;
  const long step = (long)n + 1;   // diagonal entry r sits at complex index r (n + 1)
  const long nbw = gridDim.x - (pfirst ? 1 : 0);   // the element workgroups
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < count2; i += nbw * 256) {
    const double h = G[i] - K[i];
    H[i] = h;
    s += h * h;
    if ((i & 1) == 0 && (i >> 1) % step == 0) m = fmin(m, h);
  }
  rs[threadIdx.x] = s;
  rm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rm[threadIdx.x] = fmin(rm[threadIdx.x], rm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = rs[0];
    partial[FH_MAXB + blockIdx.x] = rm[0];
  }
}

__global__ __launch_bounds__(256) void form_h_finish_kernel(const double* partial, int nb, double* h2,
                                                            double* hmin) {
  __shared__ double rs[256], rm[256];
  double s = 0.0, m = 1e300;
  for (int i = threadIdx.x; i < nb; i += 256) {
    s += partial[i];
    m = fmin(m, partial[FH_MAXB + i]);
  }
  rs[threadIdx.x] = s;
  rm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      rs[threadIdx.x] += rs[threadIdx.x + w];
      rm[threadIdx.x] = fmin(rm[threadIdx.x], rm[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *h2 = rs[0];
    *hmin = rm[0];
  }
}

hipError_t form_h(const void* G, const void* K, void* H, int n, double* partial, double* h2, double* hmin,
                  hipStream_t st, void* sweep_scratch, int* status) {
  const long c2 = 2L * n * n;
  int nb = (int)cdiv(c2, 256);
  if (nb > FH_MAXB) nb = FH_MAXB;
  if (nb < 1) nb = 1;
  // the first pivot block's inverse goes where sweep_inverse (batch 1) keeps it
  z64* pfirst = sweep_scratch ? (z64*)sweep_scratch + (long)n * n : nullptr;
  hipLaunchKernelGGL(form_h_kernel, dim3(nb + (pfirst ? 1 : 0)), dim3(256), 0, st, (const double*)G,
                     (const double*)K, (double*)H, n, c2, partial, pfirst, status);
  hipLaunchKernelGGL(form_h_finish_kernel, dim3(1), dim3(256), 0, st, (const double*)partial, nb, h2, hmin);
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
