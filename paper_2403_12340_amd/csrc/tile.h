// Complex GEMM building blocks on real 16x16x4 MFMA (f64 or f32).
//
// A complex product C = A B is run as a real product on interleaved storage:
//   C'[m][2n + c] = sum_{k, p} A'[m][2k + p] B''[2k + p][2n + c]
// where A' is A read as a real M x 2K matrix (re, im adjacent) and B'' is the
// 2K x 2N real expansion of B:
//   B''[2k][2n] = re b,  B''[2k][2n+1] = im b,  B''[2k+1][2n] = -im b,  B''[2k+1][2n+1] = re b.
// One MFMA therefore covers 16 rows x 8 complex columns x 2 complex k, and the
// result lands directly in interleaved complex layout (lane l holds real
// column l % 16, so a complex element is split over lanes l and l ^ 1).
// Conjugated operands are conjugated while staging into LDS.
//
// LDS tiles are stored k-major: As[k][m] and Bs[k][n] (complex elements) with
// a one-element pad per row.
#pragma once

#include "common.h"

namespace isdf {

template <typename T, int BM_, int BN_, int BK_, int WGM_, int WGN_>
struct Tile {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WGM = WGM_, WGN = WGN_;
  static constexpr int NT = 64 * WGM * WGN;
  static constexpr int WTM = BM / WGM, WTN = BN / WGN;
  static constexpr int FM = WTM / 16, FN = WTN / 8;
  static constexpr int LDA = BM + 1, LDB = BN + 1;
  static constexpr int AS = BK * LDA, BS = BK * LDB;  // complex elements per stage
  static_assert(WTM % 16 == 0 && WTN % 8 == 0, "wave tile must be a multiple of 16 x 8");
  static_assert(BK % 2 == 0, "BK must be even");
  typedef typename Mfma<T>::acc_t acc_t;
};

// Global -> registers -> LDS staging of one BK x BX operand tile stored [k][x].
// Source element (x, k) lives at base[x * sx + k * sk]; XCONTIG says sx == 1
// (else sk == 1).  fetch() issues every load unconditionally (out-of-range
// elements read element 0 and are masked later), keeping the raw source values
// in registers, so the loads stay in flight while the MFMA step of the previous
// tile runs; store() masks, converts to the compute type T and writes LDS.
template <typename T, typename S, int BX, int BK, int NT, bool XCONTIG>
struct Stager {
  static constexpr int E = (BX * BK + NT - 1) / NT;
  static_assert(E <= 32, "valid mask is 32 bits");
  cx<S> raw[E];
  uint32_t valid;

  __device__ __forceinline__ void fetch(const cx<S>* __restrict__ base, long sx, long sk, int x0,
                                        int k0, int X, int K, int tid) {
    valid = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = tid + e * NT;
      int x, k;
      if (XCONTIG) { x = idx % BX; k = idx / BX; } else { k = idx % BK; x = idx / BK; }
      const int gx = x0 + x, gk = k0 + k;
      const bool ok = (idx < BX * BK) && gx < X && gk < K;
      const long off = ok ? (long)gx * sx + (long)gk * sk : 0;
      raw[e] = base[off];
      valid |= (ok ? 1u : 0u) << e;
    }
  }
  __device__ __forceinline__ void store(cx<T>* lds, int ld, T csign, int tid) const {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int idx = tid + e * NT;
      if (idx >= BX * BK) break;
      int x, k;
      if (XCONTIG) { x = idx % BX; k = idx / BX; } else { k = idx % BK; x = idx / BK; }
      const bool ok = (valid >> e) & 1u;
      lds[k * ld + x] = cx<T>{ok ? (T)raw[e].re : (T)0, ok ? csign * (T)raw[e].im : (T)0};
    }
  }
};

// Expanded B staging for the single-precision kernels: each complex b is stored
// as the four floats (re, im, -im, re), i.e. both rows 2k and 2k + 1 of the real
// block form, so a lane reads its B'' element with no sign fix-up.
template <typename S, int BX, int BK, int NT>
__device__ __forceinline__ void store_b4(const Stager<float, S, BX, BK, NT, true>& sg, float* lds, int ld4,
                                         float csign, int tid) {
#pragma unroll
  for (int e = 0; e < Stager<float, S, BX, BK, NT, true>::E; ++e) {
    const int idx = tid + e * NT;
    if (idx >= BX * BK) break;
    const int x = idx % BX, k = idx / BX;
    const bool ok = (sg.valid >> e) & 1u;
    const float re = ok ? (float)sg.raw[e].re : 0.f, im = ok ? csign * (float)sg.raw[e].im : 0.f;
    *reinterpret_cast<f4*>(lds + (k * ld4 + x) * 4) = f4{re, im, -im, re};
  }
}

// One BK-deep step of the wave's FM x FN block of MFMAs on LDS tiles.
template <typename T, class TL>
__device__ __forceinline__ void tile_mma(const cx<T>* __restrict__ As, const cx<T>* __restrict__ Bs,
                                         typename TL::acc_t (&acc)[TL::FM][TL::FN], int wm0,
                                         int wn0, int lane) {
  const T* Ar = reinterpret_cast<const T*>(As);
  const T* Br = reinterpret_cast<const T*>(Bs);
  const int i = lane & 15, q = lane >> 4;
  // B'' element for this lane: k part q & 1, column part i & 1.
  const int bpart = ((q & 1) == (i & 1)) ? 0 : 1;
  const T bsign = ((q & 1) == 1 && (i & 1) == 0) ? (T)-1 : (T)1;
#pragma unroll
  for (int kk = 0; kk < TL::BK / 2; ++kk) {
    const int k = 2 * kk + (q >> 1);
    T a[TL::FM], b[TL::FN];
#pragma unroll
    for (int fm = 0; fm < TL::FM; ++fm) a[fm] = Ar[(k * TL::LDA + wm0 + fm * 16 + i) * 2 + (q & 1)];
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn) b[fn] = bsign * Br[(k * TL::LDB + wn0 + fn * 8 + (i >> 1)) * 2 + bpart];
#pragma unroll
    for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < TL::FN; ++fn) acc[fm][fn] = Mfma<T>::op(a[fm], b[fn], acc[fm][fn]);
  }
}

// The same step with B stored n-major: element (k, n) of the B tile at
// Bs[n * ldbn + k] (for operands that arrive row-major in n).
template <typename T, class TL>
__device__ __forceinline__ void tile_mma_bn(const cx<T>* __restrict__ As, const cx<T>* __restrict__ Bs, int ldbn,
                                            typename TL::acc_t (&acc)[TL::FM][TL::FN], int wm0, int wn0,
                                            int lane) {
  const T* Ar = reinterpret_cast<const T*>(As);
  const T* Br = reinterpret_cast<const T*>(Bs);
  const int i = lane & 15, q = lane >> 4;
  const int bpart = ((q & 1) == (i & 1)) ? 0 : 1;
  const T bsign = ((q & 1) == 1 && (i & 1) == 0) ? (T)-1 : (T)1;
#pragma unroll
  for (int kk = 0; kk < TL::BK / 2; ++kk) {
    const int k = 2 * kk + (q >> 1);
    T a[TL::FM], b[TL::FN];
#pragma unroll
    for (int fm = 0; fm < TL::FM; ++fm) a[fm] = Ar[(k * TL::LDA + wm0 + fm * 16 + i) * 2 + (q & 1)];
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn) b[fn] = bsign * Br[((wn0 + fn * 8 + (i >> 1)) * ldbn + k) * 2 + bpart];
#pragma unroll
    for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < TL::FN; ++fn) acc[fm][fn] = Mfma<T>::op(a[fm], b[fn], acc[fm][fn]);
  }
}

template <class TL>
__device__ __forceinline__ void zero_acc(typename TL::acc_t (&acc)[TL::FM][TL::FN]) {
#pragma unroll
  for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc[fm][fn][v] = 0;
}

// XCD-aware tile order: workgroups are dispatched round-robin over the 8 XCDs,
// so logical tiles are dealt out in contiguous runs per XCD; tiles that share
// a column block (same B panel) then run on one XCD and share its L2.
__device__ __forceinline__ int xcd_remap(int id, int total) {
  const int per = (total + 7) / 8;
  return (id % 8) * per + id / 8;
}

}  // namespace isdf
