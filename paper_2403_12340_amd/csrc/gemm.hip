// Generic complex GEMM on 16x16x4 MFMA (f64 or f32), LDS double-buffered.
//   C = alpha * diag(row_scale) * op(A) op(B) + beta * C + diag_add * I
// with an optional Hermitian mode (lower tiles only, upper written as the
// conjugate mirror).
#include "internal.h"
#include "kmajor.h"   // cu_count
#include "tile.h"

#include <algorithm>
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
  int ntm, ntn, total;
  int kchunk;   // split-K: split s covers k in [s * kchunk, (s + 1) * kchunk)
  void* part;   // split-K partial sums [split][M][N] complex (compute type), or null
  long bsa, bsb, bsc;  // batch strides (complex elements); batch item = blockIdx.z
};

template <typename T, typename SA, typename SB, typename SC, class TL, bool AMC, bool BNC>
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
  const cx<SA>* A = reinterpret_cast<const cx<SA>*>(p.A) + (long)blockIdx.z * p.bsa;
  const cx<SB>* B = reinterpret_cast<const cx<SB>*>(p.B) + (long)blockIdx.z * p.bsb;

  typename TL::acc_t acc[TL::FM][TL::FN];
  zero_acc<TL>(acc);

  const int kb = blockIdx.y * p.kchunk;
  const int ke = min(p.K, kb + p.kchunk);
  const int nk = ke > kb ? (ke - kb + TL::BK - 1) / TL::BK : 0;
  sa.fetch(A, p.sam, p.sak, m0, kb, p.M, ke, tid);
  sb.fetch(B, p.sbn, p.sbk, n0, kb, p.N, ke, tid);
  sa.store(smem, TL::LDA, (T)p.ca, tid);
  sb.store(smem + TL::AS, TL::LDB, (T)p.cb, tid);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      sa.fetch(A, p.sam, p.sak, m0, kb + (kt + 1) * TL::BK, p.M, ke, tid);
      sb.fetch(B, p.sbn, p.sbk, n0, kb + (kt + 1) * TL::BK, p.N, ke, tid);
    }
    cx<T>* sc = smem + cur * (TL::AS + TL::BS);
    cx<T>* sn = smem + (cur ^ 1) * (TL::AS + TL::BS);
    tile_mma<T, TL>(sc, sc + TL::AS, acc, wm0, wn0, lane);
    if (kt + 1 < nk) {
      sa.store(sn, TL::LDA, (T)p.ca, tid);
      sb.store(sn + TL::AS, TL::LDB, (T)p.cb, tid);
    }
    __syncthreads();
  }

  SC* Cr = reinterpret_cast<SC*>(p.C) + (long)blockIdx.z * p.bsc * 2;
  T* Pr = reinterpret_cast<T*>(p.part) + (long)blockIdx.y * p.M * p.N * 2;
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
        if (p.part) {  // raw partial sum; the reduction applies the epilogue
          if (p.herm && bm == bn && row < col) continue;
          Pr[((long)row * p.N + col) * 2 + part] = acc[fm][fn][v];
          if (p.herm && row > col) Pr[((long)col * p.N + row) * 2 + part] = part ? -acc[fm][fn][v] : acc[fm][fn][v];
          continue;
        }
        const long off = ((long)row * p.ldc + col) * 2 + part;
        double val = (double)acc[fm][fn][v];
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

// Fixed-order reduction of split-K partial sums plus the epilogue.
template <typename T, typename SC>
__global__ void splitk_reduce_kernel(GemmP p, int nsplit) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;  // real index over M N 2
  const long mn2 = (long)p.M * p.N * 2;
  if (idx >= mn2) return;
  const int part = (int)(idx & 1);
  const long e = idx >> 1;
  const int row = (int)(e / p.N), col = (int)(e % p.N);
  const T* P = reinterpret_cast<const T*>(p.part);
  double v = 0.0;
  for (int s = 0; s < nsplit; ++s) v += (double)P[(long)s * mn2 + idx];
  v *= p.alpha;
  if (p.rs) v *= p.rs[row];
  if (part == 0 && row == col) v += p.diag_add;
  SC* Cr = reinterpret_cast<SC*>(p.C);
  const long off = ((long)row * p.ldc + col) * 2 + part;
  if (p.beta != 0.0) v += p.beta * (double)Cr[off];
  if (p.herm && row == col && part == 1) v = 0.0;
  Cr[off] = (SC)v;
}

typedef Tile<double, 64, 64, 16, 2, 2> Tile64;
typedef Tile<double, 32, 32, 16, 2, 2> Tile64s;   // FP64 products too small to fill the CUs with 64x64 tiles
typedef Tile<float, 64, 64, 32, 2, 2> Tile32;

template <typename T, typename SA, typename SB, typename SC, class TL, bool AMC, bool BNC>
static hipError_t launch(const GemmDesc& d, hipStream_t st) {
  GemmP p;
  p.M = d.M; p.N = d.N; p.K = d.K;
  p.A = d.A; p.sam = d.sam; p.sak = d.sak; p.ca = d.conjA ? -1.f : 1.f;
  p.B = d.B; p.sbk = d.sbk; p.sbn = d.sbn; p.cb = d.conjB ? -1.f : 1.f;
  p.C = d.C; p.ldc = d.ldc;
  p.alpha = d.alpha; p.beta = d.beta; p.diag_add = d.diag_add; p.rs = d.row_scale;
  p.herm = d.herm ? 1 : 0;
  p.bsa = d.bsa; p.bsb = d.bsb; p.bsc = d.bsc;
  p.ntm = (int)cdiv(d.M, TL::BM);
  p.ntn = (int)cdiv(d.N, TL::BN);
  if (d.herm) p.total = p.ntm * (p.ntm + 1) / 2;
  else p.total = p.ntm * p.ntn;
  if (p.total == 0) return hipSuccess;
  int nsplit = 1;
  if (d.split_ws && d.batch == 1) {
    // enough workgroups to fill the chip, each split at least 4 K tiles deep
    nsplit = (512 + p.total - 1) / p.total;
    nsplit = std::min(nsplit, std::max(1, d.K / (4 * TL::BK)));
    nsplit = std::min(nsplit, std::max(1, d.max_split));
    const size_t need = (size_t)nsplit * d.M * d.N * 2 * sizeof(T);
    while (nsplit > 1 && (size_t)nsplit * d.M * d.N * 2 * sizeof(T) > d.split_ws_bytes) --nsplit;
    (void)need;
  }
  p.kchunk = nsplit > 1 ? (int)cdiv(cdiv(d.K, nsplit), TL::BK) * TL::BK : std::max(d.K, 1);
  nsplit = nsplit > 1 ? (int)cdiv(d.K, p.kchunk) : 1;
  p.part = nsplit > 1 ? d.split_ws : nullptr;
  const unsigned grid = 8u * (unsigned)((p.total + 7) / 8);
  hipLaunchKernelGGL((gemm_kernel<T, SA, SB, SC, TL, AMC, BNC>), dim3(grid, nsplit, std::max(d.batch, 1)),
                     dim3(TL::NT), 0, st, p);
  if (nsplit > 1) {
    const long mn2 = (long)d.M * d.N * 2;
    hipLaunchKernelGGL((splitk_reduce_kernel<T, SC>), dim3(cdiv(mn2, 256)), dim3(256), 0, st, p, nsplit);
  }
  return hipGetLastError();
}

template <typename T, typename SA, typename SB, typename SC, class TL>
static hipError_t by_layout(const GemmDesc& d, hipStream_t st) {
  const bool amc = (d.sam == 1), bnc = (d.sbn == 1);
  if (amc && bnc) return launch<T, SA, SB, SC, TL, true, true>(d, st);
  if (amc && !bnc) return launch<T, SA, SB, SC, TL, true, false>(d, st);
  if (!amc && bnc) return launch<T, SA, SB, SC, TL, false, true>(d, st);
  return launch<T, SA, SB, SC, TL, false, false>(d, st);
}

template <typename SA, typename SB, typename SC>
static hipError_t f32_types(const GemmDesc& d, hipStream_t st) {
  return by_layout<float, SA, SB, SC, Tile32>(d, st);
}

hipError_t gemm(Prec compute, const GemmDesc& d, hipStream_t st) {
  if (d.M <= 0 || d.N <= 0) return hipSuccess;
  if (d.herm && d.M != d.N) return hipErrorInvalidValue;
  if (!(d.sam == 1 || d.sak == 1) || !(d.sbk == 1 || d.sbn == 1)) return hipErrorInvalidValue;
  if (compute == P64) {
    if (d.a32 || d.b32 || d.c32) return hipErrorInvalidValue;
    // a single product with fewer 64 x 64 tiles than CUs (the N_mu x N_mu algebra) runs on
    // 32 x 32 tiles: four times the workgroups, each a quarter of the MFMA work per K step
    const long tm = cdiv(d.M, 64), tn = cdiv(d.N, 64);
    const long t64 = d.herm ? tm * (tm + 1) / 2 : tm * tn;
    if (d.batch <= 1 && !d.split_ws && t64 < cu_count())
      return by_layout<double, double, double, double, Tile64s>(d, st);
    return by_layout<double, double, double, double, Tile64>(d, st);
  }
  if (d.a32) {
    if (d.b32) return d.c32 ? f32_types<float, float, float>(d, st) : f32_types<float, float, double>(d, st);
    return d.c32 ? f32_types<float, double, float>(d, st) : f32_types<float, double, double>(d, st);
  }
  if (d.b32) return d.c32 ? f32_types<double, float, float>(d, st) : f32_types<double, float, double>(d, st);
  return d.c32 ? f32_types<double, double, float>(d, st) : f32_types<double, double, double>(d, st);
}

}  // namespace isdf
