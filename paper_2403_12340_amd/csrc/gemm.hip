// Generic complex GEMM on 16x16x4 MFMA (f64 or f32), LDS double-buffered.
//   C = alpha * diag(row_scale) * op(A) op(B) + beta * C + diag_add * I
// with an optional Hermitian mode (lower tiles only, upper written as the
// conjugate mirror) and a sweep epilogue used by the in-place HPD inverse.
#include "internal.h"
#include "tile.h"

#include <cmath>

namespace isdf {

struct GemmP {
  int M, N, K;
  const void* A; long sam, sak; float ca;
  const void* B; long sbk, sbn; float cb;
  void* C; long ldc;
  double alpha, beta, diag_add;
  const double* rs;
  int herm;
  int k0, kn; const void* R; long ldr;
  int ntm, ntn, total;
};

template <typename T, typename SA, typename SB, typename SC, class TL, bool AMC, bool BNC, bool SWEEP>
__global__ __launch_bounds__(TL::NT) void gemm_kernel(GemmP p) {
  __shared__ cx<T> smem[2 * (TL::AS + TL::BS)];
  int bm, bn;
  if (p.herm) {
    const int id = xcd_remap(blockIdx.x, p.total);
    if (id >= p.total) return;
    int r = (int)((sqrt(8.0 * id + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > id) --r;
    while ((r + 1) * (r + 2) / 2 <= id) ++r;
    bm = r;
    bn = id - r * (r + 1) / 2;
  } else {
    const int id = xcd_remap(blockIdx.x, p.total);
    if (id >= p.total) return;
    bm = id % p.ntm;
    bn = id / p.ntm;
  }
  const int m0 = bm * TL::BM, n0 = bn * TL::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % TL::WGM) * TL::WTM, wn0 = (wave / TL::WGM) * TL::WTN;

  // stage s: A at smem + s * (AS + BS), B right after it

  Stager<T, SA, TL::BM, TL::BK, TL::NT, AMC> sa;
  Stager<T, SB, TL::BN, TL::BK, TL::NT, BNC> sb;
  const cx<SA>* A = reinterpret_cast<const cx<SA>*>(p.A);
  const cx<SB>* B = reinterpret_cast<const cx<SB>*>(p.B);

  typename TL::acc_t acc[TL::FM][TL::FN];
  zero_acc<TL>(acc);

  const int nk = (p.K + TL::BK - 1) / TL::BK;
  sa.fetch(A, p.sam, p.sak, m0, 0, p.M, p.K, (T)p.ca, tid);
  sb.fetch(B, p.sbn, p.sbk, n0, 0, p.N, p.K, (T)p.cb, tid);
  sa.store(smem, TL::LDA, tid);
  sb.store(smem + TL::AS, TL::LDB, tid);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      sa.fetch(A, p.sam, p.sak, m0, (kt + 1) * TL::BK, p.M, p.K, (T)p.ca, tid);
      sb.fetch(B, p.sbn, p.sbk, n0, (kt + 1) * TL::BK, p.N, p.K, (T)p.cb, tid);
    }
    cx<T>* sc = smem + cur * (TL::AS + TL::BS);
    cx<T>* sn = smem + (cur ^ 1) * (TL::AS + TL::BS);
    tile_mma<T, TL>(sc, sc + TL::AS, acc, wm0, wn0, lane);
    if (kt + 1 < nk) {
      sa.store(sn, TL::LDA, tid);
      sb.store(sn + TL::AS, TL::LDB, tid);
    }
    __syncthreads();
  }

  SC* Cr = reinterpret_cast<SC*>(p.C);
  const int rc = lane & 15, part = rc & 1;
#pragma unroll
  for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + fm * 16 + Mfma<T>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        if (row >= p.M || col >= p.N) continue;
        const long off = ((long)row * p.ldc + col) * 2 + part;
        double val = (double)acc[fm][fn][v];
        if (SWEEP) {
          const bool rk = row >= p.k0 && row < p.k0 + p.kn;
          const bool ck = col >= p.k0 && col < p.k0 + p.kn;
          const double* R = reinterpret_cast<const double*>(p.R);
          if (rk) {
            val = R[((long)(row - p.k0) * p.ldr + col) * 2 + part];
          } else if (ck) {
            const double x = R[((long)(col - p.k0) * p.ldr + row) * 2 + part];
            val = part ? -x : x;
          } else {
            val = (double)Cr[off] - val;
          }
          Cr[off] = (SC)val;
          continue;
        }
        val *= p.alpha;
        if (p.rs) val *= p.rs[row];
        if (part == 0 && row == col) val += p.diag_add;
        if (p.beta != 0.0) val += p.beta * (double)Cr[off];
        if (p.herm && bm == bn && row < col) continue;
        if (p.herm && row == col && part == 1) val = 0.0;  // Hermitian: real diagonal
        Cr[off] = (SC)val;
        if (p.herm && row > col) Cr[((long)col * p.ldc + row) * 2 + part] = (SC)(part ? -val : val);
      }
}

typedef Tile<double, 64, 64, 16, 2, 2> Tile64;
typedef Tile<float, 64, 64, 32, 2, 2> Tile32;

template <typename T, typename SA, typename SB, typename SC, class TL, bool AMC, bool BNC, bool SW>
static hipError_t launch(const GemmDesc& d, hipStream_t st) {
  GemmP p;
  p.M = d.M; p.N = d.N; p.K = d.K;
  p.A = d.A; p.sam = d.sam; p.sak = d.sak; p.ca = d.conjA ? -1.f : 1.f;
  p.B = d.B; p.sbk = d.sbk; p.sbn = d.sbn; p.cb = d.conjB ? -1.f : 1.f;
  p.C = d.C; p.ldc = d.ldc;
  p.alpha = d.alpha; p.beta = d.beta; p.diag_add = d.diag_add; p.rs = d.row_scale;
  p.herm = d.herm ? 1 : 0;
  p.k0 = d.sw_k0; p.kn = d.sw_kn; p.R = d.R; p.ldr = d.ldr;
  p.ntm = (int)cdiv(d.M, TL::BM);
  p.ntn = (int)cdiv(d.N, TL::BN);
  if (d.herm) p.total = p.ntm * (p.ntm + 1) / 2;
  else p.total = p.ntm * p.ntn;
  if (p.total == 0) return hipSuccess;
  const unsigned grid = 8u * (unsigned)((p.total + 7) / 8);
  hipLaunchKernelGGL((gemm_kernel<T, SA, SB, SC, TL, AMC, BNC, SW>), dim3(grid), dim3(TL::NT), 0, st, p);
  return hipGetLastError();
}

template <typename T, typename SA, typename SB, typename SC, class TL, bool SW>
static hipError_t by_layout(const GemmDesc& d, hipStream_t st) {
  const bool amc = (d.sam == 1), bnc = (d.sbn == 1);
  if (amc && bnc) return launch<T, SA, SB, SC, TL, true, true, SW>(d, st);
  if (amc && !bnc) return launch<T, SA, SB, SC, TL, true, false, SW>(d, st);
  if (!amc && bnc) return launch<T, SA, SB, SC, TL, false, true, SW>(d, st);
  return launch<T, SA, SB, SC, TL, false, false, SW>(d, st);
}

template <typename SA, typename SB, typename SC>
static hipError_t f32_types(const GemmDesc& d, hipStream_t st) {
  return by_layout<float, SA, SB, SC, Tile32, false>(d, st);
}

hipError_t gemm(Prec compute, const GemmDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.herm && d.M != d.N) return hipErrorInvalidValue;
  if (!(d.sam == 1 || d.sak == 1) || !(d.sbk == 1 || d.sbn == 1)) return hipErrorInvalidValue;
  if (compute == P64) {
    if (d.a32 || d.b32 || d.c32) return hipErrorInvalidValue;
    if (d.sweep) return by_layout<double, double, double, double, Tile64, true>(d, st);
    return by_layout<double, double, double, double, Tile64, false>(d, st);
  }
  if (d.sweep) return hipErrorInvalidValue;
  if (d.a32) {
    if (d.b32) return d.c32 ? f32_types<float, float, float>(d, st) : f32_types<float, float, double>(d, st);
    return d.c32 ? f32_types<float, double, float>(d, st) : f32_types<float, double, double>(d, st);
  }
  if (d.b32) return d.c32 ? f32_types<double, float, float>(d, st) : f32_types<double, float, double>(d, st);
  return d.c32 ? f32_types<double, double, float>(d, st) : f32_types<double, double, double>(d, st);
}

}  // namespace isdf
