// Single-precision complex GEMM engine for k-major operands on gfx950 (shared
// by the pair-Gram kernel and the output GEMMs).
//
// C (M x N) += A (M x K) B (K x N) with A(m, k) at A[k * lda + m] and B(k, n) at
// B[k * ldb + n] (complex64), on f32 16x16x4 MFMA via the real block form of
// the complex product (see tile.h).  A workgroup of 8 waves owns a 128 x 64
// tile; each wave a 32 x 32 block.
#pragma once

#include "tile.h"

namespace isdf {

// A is staged as interleaved complex rows padded to 2 LDA = 32 (mod 64) floats;
// B in the expanded four-float form, rows padded to 4 LDB = 32 (mod 64) floats,
// so lanes 0-31 and 32-63 of each LDS read fall on disjoint banks.  The K loop
// is double-buffered in LDS and the fragments of the next MFMA step are read
// while the current one runs.
struct ZL {
  static constexpr int BM = 128, BN = 64, BK = 16, WGM = 4, WGN = 2, NT = 512;
  static constexpr int WTM = BM / WGM, WTN = BN / WGN, FM = WTM / 16, FN = WTN / 8;
  static constexpr int LDA = BM + 16;     // complex per A row
  static constexpr int LDB = BN + 8;      // four-float groups per B row
  static constexpr int AS = BK * LDA * 2;  // floats per A stage
  static constexpr int BS = BK * LDB * 4;  // floats per B stage
};

__device__ __forceinline__ void zl_mma(const float* __restrict__ Af, const float* __restrict__ Bf,
                                       f4 (&acc)[ZL::FM][ZL::FN], int wm0, int wn0, int lane) {
  constexpr int KK = ZL::BK / 2;
  const int i = lane & 15, q = lane >> 4;
  const float* ap = Af + ((q >> 1) * ZL::LDA + wm0 + i) * 2 + (q & 1);
  const float* bp = Bf + ((q >> 1) * ZL::LDB + wn0 + (i >> 1)) * 4 + 2 * (q & 1) + (i & 1);
  float a[2][ZL::FM], b[2][ZL::FN];
#pragma unroll
  for (int fm = 0; fm < ZL::FM; ++fm) a[0][fm] = ap[fm * 32];
#pragma unroll
  for (int fn = 0; fn < ZL::FN; ++fn) b[0][fn] = bp[fn * 32];
#pragma unroll
  for (int kk = 0; kk < KK; ++kk) {
    const int c = kk & 1;
    if (kk + 1 < KK) {
#pragma unroll
      for (int fm = 0; fm < ZL::FM; ++fm) a[c ^ 1][fm] = ap[(kk + 1) * 4 * ZL::LDA + fm * 32];
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn) b[c ^ 1][fn] = bp[(kk + 1) * 8 * ZL::LDB + fn * 32];
    }
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn) acc[fm][fn] = Mfma<float>::op(a[c][fm], b[c][fn], acc[fm][fn]);
    // issue order: the next step's LDS reads between this step's MFMAs
    if (kk + 1 < KK) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, ZL::FM * ZL::FN - 3, 0);
    }
  }
}

// Interior tiles: every K tile full, so no bounds logic at all.  Each thread
// moves two complex values per 16-byte load at offsets fixed for the whole
// kernel (only the uniform tile base advances), and the two LDS stages are
// addressed statically (the K loop is unrolled by two).
struct ZFetch {
  uint32_t aoff0, aoff1, boff;  // byte offsets of this thread's loads from the tile base
  int ax, ak, bx, bk;           // its positions in the A (16 x 128) and B (16 x 64) tiles
  f4 ra0, ra1, rb;              // staged data of one K tile
  __device__ __forceinline__ void init(int tid, long ldp, long ldb) {
    ax = 2 * (tid & 63); ak = tid >> 6; bx = 2 * (tid & 31); bk = tid >> 5;
    aoff0 = (uint32_t)((ak * ldp + ax) * 8);
    aoff1 = (uint32_t)(((ak + 8) * ldp + ax) * 8);
    boff = (uint32_t)((bk * ldb + bx) * 8);
  }
  // K tile t of the tile at (m0, n0): rows [16 t, 16 t + 16) of both k-major operands
  __device__ __forceinline__ void fetch(const c32* pm, long ldp, const c32* b, long ldb, int m0, int n0, int t) {
    const long kr = (long)t * ZL::BK;
    const char* pa = reinterpret_cast<const char*>(pm + kr * ldp + m0);
    const char* pb = reinterpret_cast<const char*>(b + kr * ldb + n0);
    ra0 = *reinterpret_cast<const f4*>(pa + aoff0);
    ra1 = *reinterpret_cast<const f4*>(pa + aoff1);
    rb = *reinterpret_cast<const f4*>(pb + boff);
  }
  // sa, sb = +1 or -1: the sign of the imaginary parts (-1 conjugates the operand)
  __device__ __forceinline__ void stage(float* buf, float sa, float sb) const {
    // A interleaved (re, sa im); B in the four-float form (re, sb im, -sb im, re)
    *reinterpret_cast<f4*>(buf + (ak * ZL::LDA + ax) * 2) = f4{ra0[0], sa * ra0[1], ra0[2], sa * ra0[3]};
    *reinterpret_cast<f4*>(buf + ((ak + 8) * ZL::LDA + ax) * 2) = f4{ra1[0], sa * ra1[1], ra1[2], sa * ra1[3]};
    float* bb = buf + ZL::AS + (bk * ZL::LDB + bx) * 4;
    const float i0 = sb * rb[1], i1 = sb * rb[3];
    *reinterpret_cast<f4*>(bb) = f4{rb[0], i0, -i0, rb[0]};
    *reinterpret_cast<f4*>(bb + 4) = f4{rb[2], i1, -i1, rb[2]};
  }
};

// Operands of one MFMA step of a K tile staged at `buf`: A at buf, B at buf + AS.
struct ZFrag {
  float a[ZL::FM], b[ZL::FN];
};
__device__ __forceinline__ void zl_frag(const float* buf, int kk, ZFrag& f, int wm0, int wn0, int lane) {
  const int i = lane & 15, q = lane >> 4;
  const float* ap = buf + ((q >> 1) * ZL::LDA + wm0 + i) * 2 + (q & 1);
  const float* bp = buf + ZL::AS + ((q >> 1) * ZL::LDB + wn0 + (i >> 1)) * 4 + 2 * (q & 1) + (i & 1);
#pragma unroll
  for (int fm = 0; fm < ZL::FM; ++fm) f.a[fm] = ap[kk * 4 * ZL::LDA + fm * 32];
#pragma unroll
  for (int fn = 0; fn < ZL::FN; ++fn) f.b[fn] = bp[kk * 8 * ZL::LDB + fn * 32];
}
__device__ __forceinline__ void zl_step(const ZFrag& f, f4 (&acc)[ZL::FM][ZL::FN]) {
#pragma unroll
  for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < ZL::FN; ++fn) acc[fm][fn] = Mfma<float>::op(f.a[fm], f.b[fn], acc[fm][fn]);
}
// issue order: the LDS reads just written in source order between the first MFMAs
__device__ __forceinline__ void zl_interleave() {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, ZL::FM * ZL::FN - 3, 0);
}

// K tiles [t0, t1) of one interior tile into the accumulator `acc`.  `z` (a
// ZFetch, or a fetch of the same interface whose B operand has another storage
// type) holds K tile t0, fetched and not yet staged, and both LDS stages are free
// on entry; or, with `staged`, K tile t0 is already in stage 0 and its first MFMA
// step's operands in f[0].  During the last K tile the loop fetches K tile nk of
// the tile at (nm0, nn0) if `refill` (the next range's first K tile), else that
// last K tile again; either way it stages what it fetched into the other stage and
// loads its first operands into f[0].  With t1 - t0 even that stage is stage 0, so
// a refilled K tile is ready for a call with `staged`.  Each kernel has a single
// instance of this loop (a kernel with two accumulators runs its ranges through
// one call site), so the loop-invariant LDS and global addresses are held once.
//
// Per K tile: steps 0 .. BK/2 - 2 (each reading the next step's operands), then the
// next K tile is staged and the barrier passed while the last step's operands are
// already in registers, so the next tile's first LDS reads overlap the last step's
// MFMAs.  Fetch, staging and barrier happen for every K tile, with no condition,
// so no path leaves loads in flight (the compiler would otherwise wait for them,
// and with them for every store issued since, before the next fetch).  Every read
// of a stage is issued before the barrier that precedes its next overwrite (the
// barrier waits for outstanding LDS operations), and the last K tile also ends
// with a barrier, so on return stage 1 is free, and stage 0 too unless the caller
// uses the staged refill.
template <class F, typename SB>
__device__ __forceinline__ void zl_range(float* smem, F& z, ZFrag (&f)[2], int t0, int t1, bool staged, float sa,
                                         float sb, const c32* A, long lda, const SB* B, long ldb, int m0, int n0,
                                         bool refill, int nm0, int nn0, int nk, f4 (&acc)[ZL::FM][ZL::FN], int wm0,
                                         int wn0, int lane) {
  constexpr int KK = ZL::BK / 2;
  if (t0 >= t1) return;
  float* s0 = smem;
  float* s1 = smem + ZL::AS + ZL::BS;
  // one K tile staged at cur, its step-0 operands in f[0]; the next one goes to nxt
  auto tile = [&](int t, const float* cur, float* nxt) {
    const bool inrange = t + 1 < t1;
    const bool other = !inrange && refill;
    z.fetch(A, lda, B, ldb, other ? nm0 : m0, other ? nn0 : n0, inrange ? t + 1 : (refill ? nk : t));
    __builtin_amdgcn_sched_barrier(0);   // the loads stay ahead of this tile's MFMAs
#pragma unroll
    for (int kk = 0; kk + 1 < KK; ++kk) {
      const int c = kk & 1;
      zl_frag(cur, kk + 1, f[c ^ 1], wm0, wn0, lane);
      zl_step(f[c], acc);
      zl_interleave();
    }
    __builtin_amdgcn_sched_barrier(0);   // and the staging (which waits for them) behind them
    z.stage(nxt, sa, sb);
    __syncthreads();
    zl_frag(nxt, 0, f[0], wm0, wn0, lane);
    zl_step(f[(KK - 1) & 1], acc);
    zl_interleave();
  };
  if (!staged) {
    z.stage(s0, sa, sb);
    __syncthreads();
    zl_frag(s0, 0, f[0], wm0, wn0, lane);
  }
  // two K tiles per pass, so both LDS stages are addressed statically
  for (int t = t0; t < t1; t += 2) {
    tile(t, s0, s1);
    if (t + 1 >= t1) break;
    tile(t + 1, s1, s0);
  }
}

// CUs of the current device (cached per device)
inline int cu_count() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) n = 256;
    cached[dev] = n;
  }
  return cached[dev];
}

}  // namespace isdf
