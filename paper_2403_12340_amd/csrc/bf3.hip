// BF16x3 split-precision pair kernel (step 1, the ISDF fit's right-hand side).
//
// Every FP32 operand value x is split into two bfloat16 parts, hi = bf16(x) and
// lo = bf16(x - hi) (round to nearest even), and a product is formed as
//   a b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi
// on 16x16x32 bf16 MFMA with FP32 accumulation (the a_lo b_lo term, of relative
// size 2^-16, is dropped).  The complex products use the real block form of
// tile.h: the grid operand is read as interleaved (re, im) rows and the point
// operand in its expanded form, two real columns per complex column.
//
// Operands are split once per build into k-tile-blocked planes, zero-padded so
// the main loop has no bounds logic:
//   A (grid):   [kt][Rpad][32] bf16, hi plane then lo plane; element (r, 2j + p)
//               of k tile kt is part p (re, im) of psi_k(r), k = 16 kt + j;
//   B (points): [kt][2 Npad][32] bf16, real column 2 mu + c holds
//               c = 0: (re, im) psi_k(r_mu),  c = 1: (-im, re) psi_k(r_mu),
//               i.e. conj(psi_k(r_mu)) in expanded form.
// k runs over the occupied states padded to a multiple of 16, then the empty
// ones, padded the same way; padded slots hold zeros.
//
// 16x16x32 bf16 MFMA lane layout (measured on gfx950): lane l supplies
// A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e = 0..7, and holds
// D[4 (l / 16) + v][l % 16] in output register v.
#include "internal.h"
#include "tile.h"

namespace isdf {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef unsigned int u4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int KSTEP = 16;   // complex states per k tile (32 real k: one MFMA step)

__device__ __forceinline__ int state_of(int k, int nv, int nc, int kvp) {
  if (k < kvp) return k < nv ? k : -1;
  const int j = k - kvp;
  return j < nc ? nv + j : -1;
}

__device__ __forceinline__ void split2(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);   // exact difference in FP32
}

// One thread per (grid row r, k tile): 16 states, written as 64 bytes per plane.
__global__ __launch_bounds__(256) void split_rows_kernel(const z64* __restrict__ psi, long ld, long nr,
                                                         int nv, int nc, int kvp, long rpad,
                                                         bf8* __restrict__ hi, bf8* __restrict__ lo) {
  const long r = (long)blockIdx.x * 256 + threadIdx.x;
  const int kt = blockIdx.y;
  if (r >= rpad) return;
  bf8 h[4], l[4];
#pragma unroll
  for (int j = 0; j < KSTEP; ++j) {
    const int n = state_of(kt * KSTEP + j, nv, nc, kvp);
    z64 v = {0.0, 0.0};
    if (n >= 0 && r < nr) v = psi[(long)n * ld + r];
    __bf16 a, b, c, d;
    split2((float)v.re, a, b);
    split2((float)v.im, c, d);
    h[j >> 2][(2 * j) & 7] = a;
    l[j >> 2][(2 * j) & 7] = b;
    h[j >> 2][(2 * j + 1) & 7] = c;
    l[j >> 2][(2 * j + 1) & 7] = d;
  }
  const long o = ((long)kt * rpad + r) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hi[o + q] = h[q];
    lo[o + q] = l[q];
  }
}

// One thread per (point mu, k tile): two expanded real columns per plane.
__global__ __launch_bounds__(64) void split_points_kernel(const z64* __restrict__ pm, long ld, int nmu, int nv,
                                                          int nc, int kvp, long cpad, bf8* __restrict__ hi,
                                                          bf8* __restrict__ lo) {
  const int mu = blockIdx.x * 64 + threadIdx.x;
  const int kt = blockIdx.y;
  if (2L * mu >= cpad) return;
  bf8 h0[4], l0[4], h1[4], l1[4];
#pragma unroll
  for (int j = 0; j < KSTEP; ++j) {
    const int n = state_of(kt * KSTEP + j, nv, nc, kvp);
    z64 v = {0.0, 0.0};
    if (n >= 0 && mu < nmu) v = pm[(long)n * ld + mu];
    __bf16 rh, rl, ih, il;
    split2((float)v.re, rh, rl);
    split2((float)v.im, ih, il);
    const int q = j >> 2, e = (2 * j) & 7;
    h0[q][e] = rh; l0[q][e] = rl; h0[q][e + 1] = ih; l0[q][e + 1] = il;     // (re, im)
    h1[q][e] = -ih; l1[q][e] = -il; h1[q][e + 1] = rh; l1[q][e + 1] = rl;   // (-im, re)
  }
  const long o0 = ((long)kt * cpad + 2L * mu) * 4, o1 = o0 + 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hi[o0 + q] = h0[q]; lo[o0 + q] = l0[q];
    hi[o1 + q] = h1[q]; lo[o1 + q] = l1[q];
  }
}

// Tile: 128 grid rows x 64 points (128 real columns); 4 waves in 2 x 2, each
// 64 rows x 64 real columns (4 x 4 MFMA blocks).  An LDS stage holds one k tile
// of the four planes (A hi, A lo, B hi, B lo; 8 KB each, 64 bytes per row);
// the 16-byte chunk g of row i sits at chunk g ^ ((i >> 1) & 3) so that the
// eight lanes of each LDS access phase hit distinct banks.
struct BT {
  static constexpr int BM = 128, BNR = 128, NT = 256;
  static constexpr int PLANE = 8192, STAGE = 4 * PLANE;
};

__device__ __forceinline__ int swz(int row, int g) { return row * 64 + ((g ^ ((row >> 1) & 3)) << 4); }

__device__ __forceinline__ void bf3_mma(const char* __restrict__ buf, f4 (&acc)[4][4], int wm, int wn, int lane) {
  const int i = lane & 15, g = lane >> 4;
  const char* pa = buf + swz(wm * 64 + i, g);
  const char* pb = buf + 2 * BT::PLANE + swz(wn * 64 + i, g);
  bf8 a[4], bh[4], bl[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    a[f] = *reinterpret_cast<const bf8*>(pa + f * 1024);
    bh[f] = *reinterpret_cast<const bf8*>(pb + f * 1024);
    bl[f] = *reinterpret_cast<const bf8*>(pb + BT::PLANE + f * 1024);
  }
  // a_hi b_hi + a_hi b_lo, then a_lo b_hi (a_lo loaded into a_hi's registers)
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], bh[fn], acc[fm][fn], 0, 0, 0);
#pragma unroll
  for (int fm = 0; fm < 4; ++fm) {
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], bl[fn], acc[fm][fn], 0, 0, 0);
    a[fm] = *reinterpret_cast<const bf8*>(pa + BT::PLANE + fm * 1024);
  }
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], bh[fn], acc[fm][fn], 0, 0, 0);
}

// out[mu][r] = conj(P(r, mu)) Q(r, mu) (complex64, row stride ldo) with
// P = sum over occupied k tiles, Q over empty ones.  The tiles of one grid-row
// block (all point blocks) are consecutive in each XCD's share, so the block's
// grid rows are read from HBM once per XCD.
__global__ __launch_bounds__(BT::NT) __attribute__((amdgpu_waves_per_eu(2))) void zpair_bf3_kernel(const char* __restrict__ A, long aplane,
                                                          const char* __restrict__ B, long bplane, long rpad,
                                                          long cpad, int ktv, int kt, float* __restrict__ out,
                                                          long ldo, long nr, int nmu, int ntn, int total) {
  __shared__ __attribute__((aligned(16))) char smem[2 * BT::STAGE];
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  const int bn = id % ntn, bm = id / ntn;
  const long r0 = (long)bm * BT::BM, c0 = (long)bn * BT::BNR;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 1, wn = wave >> 1;
  // this thread's two 16-byte chunks of every plane tile: global (unswizzled) and LDS offsets
  const int q0 = tid, q1 = tid + BT::NT;
  const int s0 = swz(q0 >> 2, q0 & 3), s1 = swz(q1 >> 2, q1 & 3);
  u4 st[8];
  auto gload = [&](int t) {
    const char* pa = A + ((long)t * rpad + r0) * 64;
    const char* pb = B + ((long)t * cpad + c0) * 64;
    st[0] = *reinterpret_cast<const u4*>(pa + q0 * 16);
    st[1] = *reinterpret_cast<const u4*>(pa + q1 * 16);
    st[2] = *reinterpret_cast<const u4*>(pa + aplane + q0 * 16);
    st[3] = *reinterpret_cast<const u4*>(pa + aplane + q1 * 16);
    st[4] = *reinterpret_cast<const u4*>(pb + q0 * 16);
    st[5] = *reinterpret_cast<const u4*>(pb + q1 * 16);
    st[6] = *reinterpret_cast<const u4*>(pb + bplane + q0 * 16);
    st[7] = *reinterpret_cast<const u4*>(pb + bplane + q1 * 16);
  };
  auto lstore = [&](char* buf) {
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      *reinterpret_cast<u4*>(buf + p * BT::PLANE + s0) = st[2 * p];
      *reinterpret_cast<u4*>(buf + p * BT::PLANE + s1) = st[2 * p + 1];
    }
  };
  f4 accp[4][4], accq[4][4];
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) accp[fm][fn] = accq[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
  gload(0);
  lstore(smem);
  __syncthreads();
  // occupied k tiles into P, then the empty ones into Q (two loops, so each
  // accumulator stays in its registers)
  for (int t = 0; t < ktv; ++t) {
    if (t + 1 < kt) gload(t + 1);
    bf3_mma(smem + (t & 1) * BT::STAGE, accp, wm, wn, lane);
    if (t + 1 < kt) lstore(smem + ((t + 1) & 1) * BT::STAGE);
    __syncthreads();
  }
  for (int t = ktv; t < kt; ++t) {
    if (t + 1 < kt) gload(t + 1);
    bf3_mma(smem + (t & 1) * BT::STAGE, accq, wm, wn, lane);
    if (t + 1 < kt) lstore(smem + ((t + 1) & 1) * BT::STAGE);
    __syncthreads();
  }
  // epilogue: lane (i, g) holds rows 4g + v of real column i of each block; the
  // two halves of a complex value sit in lanes i, i ^ 1.  After one exchange the
  // even lane stores rows 4g, 4g + 1 and the odd lane rows 4g + 2, 4g + 3, each
  // as one 16-byte (two complex64) store when aligned and in range.
  const int i = lane & 15, g = lane >> 4, part = i & 1;
  const bool vec_ok = (ldo & 1) == 0;
#pragma unroll
  for (int fm = 0; fm < 4; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
      float val[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float po = accp[fm][fn][v], qo = accq[fm][fn][v];
        const float px = xor1(po), qx = xor1(qo);
        val[v] = part == 0 ? (po * qo + px * qx) : (px * qo - po * qx);
      }
      const float y0 = xor1(part == 0 ? val[2] : val[0]);
      const float y1 = xor1(part == 0 ? val[3] : val[1]);
      const int mu = (int)((c0 + wn * 64 + fn * 16 + i) >> 1);
      const long r = r0 + wm * 64 + fm * 16 + 4 * g + 2 * part;   // first of this lane's two rows
      if (mu >= nmu) continue;
      const f4 w = part == 0 ? f4{val[0], y0, val[1], y1} : f4{y0, val[2], y1, val[3]};
      float* o = out + ((long)mu * ldo + r) * 2;
      if (vec_ok && r + 1 < nr) {
        *reinterpret_cast<f4*>(o) = w;
      } else {
        if (r < nr) { o[0] = w[0]; o[1] = w[1]; }
        if (r + 1 < nr) { o[2] = w[2]; o[3] = w[3]; }
      }
    }
}

}  // namespace

size_t bf3_rows_bytes(long nr, int nv, int nc) {
  const long kt = (bf3_pad(nv) + bf3_pad(nc)) / KSTEP;
  return (size_t)2 * kt * bf3_rpad(nr) * 64;
}

size_t bf3_points_bytes(int nmu, int nv, int nc) {
  const long kt = (bf3_pad(nv) + bf3_pad(nc)) / KSTEP;
  return (size_t)2 * kt * 2 * bf3_npad(nmu) * 64;
}

hipError_t bf3_split_rows(const void* psi, long ld, long nr, int nv, int nc, void* planes, hipStream_t st) {
  const int kvp = bf3_pad(nv);
  const int kt = (kvp + bf3_pad(nc)) / KSTEP;
  const long rpad = bf3_rpad(nr);
  bf8* hi = reinterpret_cast<bf8*>(planes);
  bf8* lo = hi + (long)kt * rpad * 4;
  hipLaunchKernelGGL(split_rows_kernel, dim3(cdiv(rpad, 256), kt), dim3(256), 0, st, (const z64*)psi, ld, nr, nv,
                     nc, kvp, rpad, hi, lo);
  return hipGetLastError();
}

hipError_t bf3_split_points(const void* pm, long ld, int nmu, int nv, int nc, void* planes, hipStream_t st) {
  const int kvp = bf3_pad(nv);
  const int kt = (kvp + bf3_pad(nc)) / KSTEP;
  const long cpad = 2L * bf3_npad(nmu);
  bf8* hi = reinterpret_cast<bf8*>(planes);
  bf8* lo = hi + (long)kt * cpad * 4;
  hipLaunchKernelGGL(split_points_kernel, dim3(cdiv(cpad / 2, 64), kt), dim3(64), 0, st, (const z64*)pm, ld, nmu,
                     nv, nc, kvp, cpad, hi, lo);
  return hipGetLastError();
}

hipError_t zpair_bf3(long nr, int nmu, int nv, int nc, const void* rows, const void* points, void* out, long ldo,
                     hipStream_t st) {
  const int kvp = bf3_pad(nv);
  const int ktv = kvp / KSTEP, kt = (kvp + bf3_pad(nc)) / KSTEP;
  const long rpad = bf3_rpad(nr), cpad = 2L * bf3_npad(nmu);
  const long ntm = rpad / BT::BM, ntn = cpad / BT::BNR;
  const long total = ntm * ntn;
  if (total == 0) return hipSuccess;
  if (total > 0x7fffffffL / 8) return hipErrorInvalidValue;
  const unsigned grid = 8u * (unsigned)((total + 7) / 8);
  const long aplane = (long)kt * rpad * 64, bplane = (long)kt * cpad * 64;
  hipLaunchKernelGGL(zpair_bf3_kernel, dim3(grid), dim3(BT::NT), 0, st, (const char*)rows, aplane,
                     (const char*)points, bplane, rpad, cpad, ktv, kt, (float*)out, ldo, nr, nmu, (int)ntn,
                     (int)total);
  return hipGetLastError();
}

}  // namespace isdf
