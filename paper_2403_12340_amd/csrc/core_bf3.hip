// Core M = f C Omega^{-1} C^H (eq. COmegaCstar) in the BF16x3 mode.
//
// Each FP32 operand value x is split as hi = bf16(x), lo = bf16(x - hi) (round
// to nearest even) and a product is a_hi b_hi + a_hi b_lo + a_lo b_hi on the
// 16x16x32 bf16 MFMA with FP32 accumulation, as in the BF16x3 pair kernel
// (bf3.hip), whose lane layout and LDS swizzle this kernel shares.  Operand
// planes in LDS, per k tile of 16 complex states (32 real k):
//   A planes: [128 rows][32] bf16, element (m, 2j + p) = part p (re, im) of A(m, j);
//   B planes: [128 real columns][32] bf16, real column 2n holds (br, -bi) and real
//             column 2n + 1 holds (bi, br) of b = B(j, n) along each j, so the real
//             product of an A row with the two columns gives the real and the
//             imaginary part of the complex product.
#include "internal.h"
#include "tile.h"

#include <algorithm>

namespace isdf {

typedef __bf16 bf8g __attribute__((ext_vector_type(8)));
typedef unsigned int u4g __attribute__((ext_vector_type(4)));

namespace {

constexpr int KT = 16;      // complex k per tile (one 32-deep bf16 MFMA step)
constexpr int GBM = 128;    // complex rows per tile
constexpr int GBN = 64;     // complex columns per tile (128 real)
constexpr int PLANE = 8192; // bytes of one plane's k tile in LDS (128 rows x 64 B)
constexpr int STAGE = 4 * PLANE;

__device__ __forceinline__ void split2(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);   // exact difference in FP32
}

// A planes: one thread per (row m, k tile); the source is complex64 or complex128.
// With `copy`, the values also go to copy[k ld + m] as complex64.
template <typename S>
__global__ __launch_bounds__(256) void split_arows_kernel(const cx<S>* __restrict__ s, long ld, int M, int K,
                                                          float sgn, long mpad, bf8g* __restrict__ hi,
                                                          bf8g* __restrict__ lo, c32* __restrict__ copy) {
  const long m = (long)blockIdx.x * 256 + threadIdx.x;
  const int kt = blockIdx.y;
  if (m >= mpad) return;
  bf8g h[4], l[4];
#pragma unroll
  for (int j = 0; j < KT; ++j) {
    const int k = kt * KT + j;
    float vr = 0.f, vi = 0.f;
    if (m < M && k < K) {
      const cx<S> v = s[(long)k * ld + m];
      vr = (float)v.re;
      vi = (float)v.im;
      if (copy) copy[(long)k * ld + m] = c32{vr, vi};
    }
    __bf16 a, b, c, d;
    split2(vr, a, b);
    split2(sgn * vi, c, d);
    h[j >> 2][(2 * j) & 7] = a;
    l[j >> 2][(2 * j) & 7] = b;
    h[j >> 2][(2 * j + 1) & 7] = c;
    l[j >> 2][(2 * j + 1) & 7] = d;
  }
  const long o = ((long)kt * mpad + m) * 4;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    hi[o + q] = h[q];
    lo[o + q] = l[q];
  }
}

// the 16-byte chunk g of LDS row i sits at chunk g ^ ((i >> 1) & 3): the eight lanes
// of each LDS access phase hit distinct banks
__device__ __forceinline__ int swz(int row, int g) { return row * 64 + ((g ^ ((row >> 1) & 3)) << 4); }

// lower-triangle tile list of a square (128-row) x (64-column) tile grid, row-major:
// row bm holds the tiles bn <= 2 bm + 1
__device__ __forceinline__ void herm_tile_bf3(int id, int& bm, int& bn) {
  int r = (int)((sqrtf(4.f * (float)id + 1.f) - 1.f) * 0.5f);
  while (r * (r + 1) > id) --r;
  while ((r + 1) * (r + 2) <= id) ++r;
  bm = r;
  bn = id - r * (r + 1);
}

// ---- core M = f C Omega^{-1} C^H in BF16x3 (eq. COmegaCstar) ---------------------------
// The structure of the single-precision core (core32.hip): for each occupied i,
// G_i = B diag(w_i) B^H over the empty states j, with A(mu, j) = b_j(mu) (the same
// for every i: split once into A planes) and B(j, nu) = w_ij conj(b_j(nu)) (split
// while staged, from a complex64 copy of the samples made with the A planes, and the
// FP64 weights); G_i accumulates in FP32 over
// the Nc terms and the rank-one factor conj(a_i(mu)) a_i(nu) is applied in FP64
// registers after each i.  8 waves (4 x 2), each 32 rows x 64 real columns of a
// 128 x 64 lower-triangle tile; the occupied index is split across workgroups and
// the partial sums added by core_reduce.
constexpr int CNT = 512;

__device__ __forceinline__ void mma3_8w(const char* __restrict__ buf, f4 (&acc)[2][4], int wm, int wn, int lane) {
  const int i = lane & 15, g = lane >> 4;
  const char* pa = buf + swz(wm * 32 + i, g);
  const char* pb = buf + 2 * PLANE + swz(wn * 64 + i, g);
  bf8g a[2], bh[4], bl[4];
#pragma unroll
  for (int f = 0; f < 2; ++f) a[f] = *reinterpret_cast<const bf8g*>(pa + f * 1024);
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    bh[f] = *reinterpret_cast<const bf8g*>(pb + f * 1024);
    bl[f] = *reinterpret_cast<const bf8g*>(pb + PLANE + f * 1024);
  }
#pragma unroll
  for (int fm = 0; fm < 2; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], bh[fn], acc[fm][fn], 0, 0, 0);
#pragma unroll
  for (int fm = 0; fm < 2; ++fm) {
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], bl[fn], acc[fm][fn], 0, 0, 0);
    a[fm] = *reinterpret_cast<const bf8g*>(pa + PLANE + fm * 1024);
  }
#pragma unroll
  for (int fm = 0; fm < 2; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) acc[fm][fn] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[fm], bh[fn], acc[fm][fn], 0, 0, 0);
}

__device__ __forceinline__ void core_tile_bf3(int id, int& bm, int& bn) { herm_tile_bf3(id, bm, bn); }

__device__ __forceinline__ z64 conj_mul(z64 a, z64 b) {   // conj(a) b
  return z64{a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}

__global__ __launch_bounds__(CNT) void core_bf3_kernel(int nmu, int nv, int nc, const z64* __restrict__ pm,
                                                       const char* __restrict__ A, long aplane,
                                                       const double* __restrict__ w, c32* __restrict__ part,
                                                       int nsplit, int total) {
  __shared__ __attribute__((aligned(16))) char smem[2 * STAGE];
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  int bm, bn;
  core_tile_bf3(id, bm, bn);
  const int m0 = bm * GBM, n0 = bn * GBN;
  const int split = blockIdx.y;
  w += (long)blockIdx.z * nv * nc;                        // weight set of this batch item
  part += (long)blockIdx.z * nsplit * nmu * nmu;
  const int i0 = (int)((long)split * nv / nsplit), i1 = (int)((long)(split + 1) * nv / nsplit);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave & 3, wn = wave >> 2;
  const int li = lane & 15, g = lane >> 4, pp = li & 1;
  const c32* pc = reinterpret_cast<const c32*>(A + 2 * aplane);   // empty states at the points (complex64), [j][mu]
  const int nt = nc / KT;
  const int S = (i1 - i0) * nt;
  // A (pre-split planes): this thread's 16-byte chunk of the hi and of the lo plane
  const int sa = swz(tid >> 2, tid & 3);
  // B (split here): complex column c of the tile, states 2p, 2p + 1 of the k tile
  const int bc = tid & 63, bp = tid >> 6;
  const int sb0 = swz(2 * bc, bp >> 1) + (bp & 1) * 8, sb1 = swz(2 * bc + 1, bp >> 1) + (bp & 1) * 8;
  u4g ra[2];
  c32 rb[2];
  double rw[2];
  auto gload = [&](int s) {
    const int i = i0 + s / nt, t = s % nt;
    const char* pa = A + ((long)t * ((long)nmu) + m0) * 64;
    ra[0] = *reinterpret_cast<const u4g*>(pa + tid * 16);
    ra[1] = *reinterpret_cast<const u4g*>(pa + aplane + tid * 16);
    const int j = t * KT + 2 * bp;
    rb[0] = pc[(long)j * nmu + n0 + bc];
    rb[1] = pc[(long)(j + 1) * nmu + n0 + bc];
    rw[0] = w[(long)i * nc + j];
    rw[1] = w[(long)i * nc + j + 1];
  };
  auto stage = [&](char* buf) {
    *reinterpret_cast<u4g*>(buf + sa) = ra[0];
    *reinterpret_cast<u4g*>(buf + PLANE + sa) = ra[1];
    // B(j, nu) = w conj(b): (Br, Bi) = (w br, -w bi); column 2c: (Br, -Bi), column 2c + 1: (Bi, Br)
    __bf16 h0[4], l0[4], h1[4], l1[4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const float br = (float)(rw[q] * (double)rb[q].re), bi = (float)(-rw[q] * (double)rb[q].im);
      __bf16 rh, rl, ih, il, nh, nl;
      split2(br, rh, rl);
      split2(bi, ih, il);
      split2(-bi, nh, nl);
      h0[2 * q] = rh; l0[2 * q] = rl; h0[2 * q + 1] = nh; l0[2 * q + 1] = nl;
      h1[2 * q] = ih; l1[2 * q] = il; h1[2 * q + 1] = rh; l1[2 * q + 1] = rl;
    }
    typedef __bf16 bf4 __attribute__((ext_vector_type(4)));
    *reinterpret_cast<bf4*>(buf + 2 * PLANE + sb0) = bf4{h0[0], h0[1], h0[2], h0[3]};
    *reinterpret_cast<bf4*>(buf + 3 * PLANE + sb0) = bf4{l0[0], l0[1], l0[2], l0[3]};
    *reinterpret_cast<bf4*>(buf + 2 * PLANE + sb1) = bf4{h1[0], h1[1], h1[2], h1[3]};
    *reinterpret_cast<bf4*>(buf + 3 * PLANE + sb1) = bf4{l1[0], l1[1], l1[2], l1[3]};
  };
  f4 acc[2][4];
  double acc64[2][4][4];
#pragma unroll
  for (int fm = 0; fm < 2; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) {
      acc[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[fm][fn][v] = 0.0;
    }
  // acc64 += conj(a_i(mu)) a_i(nu) G_i for this lane's elements, then G_i restarts
  auto flush = [&](int i) {
    const z64* ai = pm + (long)i * nmu;
    z64 an[4];
#pragma unroll
    for (int fn = 0; fn < 4; ++fn) an[fn] = ai[n0 + ((wn * 64 + fn * 16 + li) >> 1)];
#pragma unroll
    for (int fm = 0; fm < 2; ++fm)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const z64 am = ai[m0 + wm * 32 + fm * 16 + 4 * g + v];
#pragma unroll
        for (int fn = 0; fn < 4; ++fn) {
          const float self = acc[fm][fn][v], other = xor1(self);
          const double gr = pp ? other : self, gi = pp ? self : other;
          const z64 t = conj_mul(am, an[fn]);
          acc64[fm][fn][v] += pp ? t.re * gi + t.im * gr : t.re * gr - t.im * gi;
          acc[fm][fn][v] = 0.f;
        }
      }
  };
  if (S > 0) {
    gload(0);
    stage(smem);
  }
  __syncthreads();
  for (int s = 0; s < S; ++s) {
    if (s + 1 < S) gload(s + 1);
    mma3_8w(smem + (s & 1) * STAGE, acc, wm, wn, lane);
    if (s + 1 < S) stage(smem + ((s + 1) & 1) * STAGE);
    __syncthreads();
    if (s % nt == nt - 1) flush(i0 + s / nt);
  }
  float* out = reinterpret_cast<float*>(part + (long)split * nmu * nmu);
#pragma unroll
  for (int fm = 0; fm < 2; ++fm)
#pragma unroll
    for (int fn = 0; fn < 4; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm * 32 + fm * 16 + 4 * g + v;
        const int col = n0 + ((wn * 64 + fn * 16 + li) >> 1);
        if (row < col) continue;
        const float val = (row == col && pp == 1) ? 0.f : (float)acc64[fm][fn][v];   // Hermitian: real diagonal
        out[((long)row * nmu + col) * 2 + pp] = val;
        if (row > col) out[((long)col * nmu + row) * 2 + pp] = pp ? -val : val;
      }
}

}  // namespace

bool core_bf3_fits(int nmu, int nc) { return nmu >= GBM && nmu % GBM == 0 && nc >= KT && nc % KT == 0; }

// the hi and lo planes, then a complex64 copy of the empty states at the points (the B
// operand's source: half the bytes per k tile of the complex128 samples)
size_t core_bf3_plane_bytes(int nmu, int nc) { return (size_t)2 * (nc / KT) * nmu * 64 + (size_t)nc * nmu * 8; }

hipError_t core_bf3_split(int nmu, int nv, int nc, const void* pm, void* planes, hipStream_t st) {
  if (!core_bf3_fits(nmu, nc)) return hipErrorInvalidValue;
  const int kt = nc / KT;
  bf8g* hi = reinterpret_cast<bf8g*>(planes);
  bf8g* lo = hi + (long)kt * nmu * 4;
  c32* copy = reinterpret_cast<c32*>(lo + (long)kt * nmu * 4);
  hipLaunchKernelGGL(split_arows_kernel<double>, dim3(cdiv(nmu, 256), kt), dim3(256), 0, st,
                     (const z64*)pm + (long)nv * nmu, (long)nmu, nmu, nc, 1.f, (long)nmu, hi, lo, copy);
  return hipGetLastError();
}

hipError_t core_bf3_partial(int nmu, int nv, int nc, const void* pm, const void* planes, const double* w,
                            void* part, int nsplit, hipStream_t st, int batch) {
  if (!core_bf3_fits(nmu, nc) || nsplit < 1 || nsplit > nv) return hipErrorInvalidValue;
  const int nti = nmu / GBM, total = nti * (nti + 1);
  const unsigned gx = 8u * (unsigned)((total + 7) / 8);
  const long aplane = (long)(nc / KT) * nmu * 64;
  hipLaunchKernelGGL(core_bf3_kernel, dim3(gx, nsplit, batch), dim3(CNT), 0, st, nmu, nv, nc, (const z64*)pm,
                     (const char*)planes, aplane, w, (c32*)part, nsplit, total);
  return hipGetLastError();
}

}  // namespace isdf
