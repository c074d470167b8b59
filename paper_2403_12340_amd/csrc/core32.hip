// Core M = f C Omega^{-1} C^H (eq. COmegaCstar) in the single-precision modes, on
// the k-major MFMA engine of kmajor.h.
//
// With a_i = psi_i(r_mu) (occupied) and b_j = psi_j(r_mu) (empty) at the points,
// and w_ij the pair weight,
//   M(mu, nu) = f sum_i conj(a_i(mu)) a_i(nu) G_i(mu, nu),
//   G_i = B diag(w_i) B^H,  G_i(mu, nu) = sum_j b_j(mu) w_ij conj(b_j(nu)).
// Each G_i is a k-major complex GEMM over the empty states (A(mu, j) = b_j(mu),
// B(j, nu) = w_ij conj(b_j(nu)): the weight is one scalar per staged B row), with
// FP32 accumulation over the Nc terms; the rank-one factor conj(a_i) a_i^T is
// applied to the accumulators in FP64 and summed over i in FP64 registers.  A
// workgroup owns one 128 x 64 tile of the lower triangle and a contiguous range of
// i; the partial sums of the ranges are added by core_reduce.  Operands come
// straight from the FP64 point samples and are rounded to FP32 while staged.
#include "internal.h"
#include "kmajor.h"

#include <algorithm>

namespace isdf {

namespace {

// lower-triangle tile list of a square (nti 128-row) x (2 nti 64-column) grid,
// row-major: row bm holds the tiles bn <= 2 bm + 1
__device__ __forceinline__ void core_tile(int id, int& bm, int& bn) {
  int r = (int)((sqrtf(4.f * (float)id + 1.f) - 1.f) * 0.5f);
  while (r * (r + 1) > id) --r;
  while ((r + 1) * (r + 2) <= id) ++r;
  bm = r;
  bn = id - r * (r + 1);
}

// One K tile (16 empty states) of G_i: each thread loads two FP64 complex values
// of A rows ak and ak + 8 and of B row bk (32-byte loads at fixed offsets from
// the uniform tile base), plus the weight of its B row.
struct CFetch {
  uint32_t aoff0, aoff1, boff;
  int ax, ak, bx, bk;
  d4 ra0, ra1, rb;
  double wr;
  __device__ __forceinline__ void init(int tid, long ld) {
    ax = 2 * (tid & 63); ak = tid >> 6; bx = 2 * (tid & 31); bk = tid >> 5;
    aoff0 = (uint32_t)((ak * ld + ax) * 16);
    aoff1 = (uint32_t)(((ak + 8) * ld + ax) * 16);
    boff = (uint32_t)((bk * ld + bx) * 16);
  }
  // K tile t of the empty-state samples pc ([j][mu], leading dimension ld) for weights wi
  __device__ __forceinline__ void fetch(const z64* pc, long ld, const double* wi, int m0, int n0, int t) {
    const long kr = (long)t * ZL::BK;
    const char* pa = reinterpret_cast<const char*>(pc + kr * ld + m0);
    const char* pb = reinterpret_cast<const char*>(pc + kr * ld + n0);
    ra0 = *reinterpret_cast<const d4*>(pa + aoff0);
    ra1 = *reinterpret_cast<const d4*>(pa + aoff1);
    rb = *reinterpret_cast<const d4*>(pb + boff);
    wr = wi[kr + bk];
  }
  // A interleaved (re, im); B = w conj(b) in the four-float form (re, im, -im, re)
  __device__ __forceinline__ void stage(float* buf) const {
    *reinterpret_cast<f4*>(buf + (ak * ZL::LDA + ax) * 2) =
        f4{(float)ra0[0], (float)ra0[1], (float)ra0[2], (float)ra0[3]};
    *reinterpret_cast<f4*>(buf + ((ak + 8) * ZL::LDA + ax) * 2) =
        f4{(float)ra1[0], (float)ra1[1], (float)ra1[2], (float)ra1[3]};
    float* bb = buf + ZL::AS + (bk * ZL::LDB + bx) * 4;
    const float re0 = (float)(wr * rb[0]), im0 = (float)(-wr * rb[1]);
    const float re1 = (float)(wr * rb[2]), im1 = (float)(-wr * rb[3]);
    *reinterpret_cast<f4*>(bb) = f4{re0, im0, -im0, re0};
    *reinterpret_cast<f4*>(bb + 4) = f4{re1, im1, -im1, re1};
  }
};

__global__ __launch_bounds__(ZL::NT) void core32_kernel(int nmu, int nv, int nc, const z64* __restrict__ pm,
                                                        const double* __restrict__ w, c32* __restrict__ part,
                                                        int nsplit, int total) {
  __shared__ float smem[2 * (ZL::AS + ZL::BS)];
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  int bm, bn;
  core_tile(id, bm, bn);
  const int m0 = bm * ZL::BM, n0 = bn * ZL::BN;
  const int split = blockIdx.y;
  w += (long)blockIdx.z * nv * nc;                        // weight set of this batch item
  part += (long)blockIdx.z * nsplit * nmu * nmu;
  const int i0 = (int)((long)split * nv / nsplit), i1 = (int)((long)(split + 1) * nv / nsplit);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % ZL::WGM) * ZL::WTM, wn0 = (wave / ZL::WGM) * ZL::WTN;
  const int rc = lane & 15, pp = rc & 1;
  const z64* pc = pm + (long)nv * nmu;
  const int nt = nc / ZL::BK;                 // even (nc % 32 == 0)
  const int S = (i1 - i0) * nt;

  f4 acc[ZL::FM][ZL::FN];
  double acc64[ZL::FM][ZL::FN][4];
#pragma unroll
  for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < ZL::FN; ++fn) {
      acc[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[fm][fn][v] = 0.0;
    }
  z64 am[ZL::FM][4], an[ZL::FN];   // a_i at this lane's rows and columns
  auto load_a = [&](int i) {
    const z64* ai = pm + (long)i * nmu;
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int v = 0; v < 4; ++v) am[fm][v] = ai[m0 + wm0 + fm * 16 + Mfma<float>::row(lane, v)];
#pragma unroll
    for (int fn = 0; fn < ZL::FN; ++fn) an[fn] = ai[n0 + wn0 + fn * 8 + (rc >> 1)];
  };
  // acc64 += conj(a_i(mu)) a_i(nu) G_i; a complex element sits in lanes l, l ^ 1
  auto flush = [&]() {
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float self = acc[fm][fn][v], other = xor1(self);
          const double gr = pp ? other : self, gi = pp ? self : other;
          const z64 t = cmulc(am[fm][v], an[fn]);
          acc64[fm][fn][v] += pp ? t.re * gi + t.im * gr : t.re * gr - t.im * gi;
          acc[fm][fn][v] = 0.f;
        }
  };
  float* buf0 = smem;
  float* buf1 = smem + ZL::AS + ZL::BS;
  CFetch cf;
  cf.init(tid, nmu);
  auto fetch_step = [&](int s) { cf.fetch(pc, nmu, w + (long)(i0 + s / nt) * nc, m0, n0, s % nt); };
  // One K tile (step s of the flattened (state, K tile) walk) staged at cur, its first MFMA
  // step's operands in f[0]: MFMA steps 0 .. BK/2 - 2, then the next K tile is staged and
  // the barrier passed before the last step (its operands already in registers), so the
  // next tile's first LDS reads overlap it.  After a state's last K tile its G_i goes
  // into the FP64 sums.
  ZFrag f[2];
  // The fetch, staging and barrier happen for every K tile (the last one fetches itself
  // again into the free stage), so no path leaves loads in flight for the compiler to
  // wait on before the next fetch; scheduling barriers keep the loads at the top of the
  // tile and the staging behind the MFMA steps.
  auto tile = [&](int s, const float* cur, float* nxt) {
    constexpr int KK = ZL::BK / 2;
    const bool end = s % nt == nt - 1;
    fetch_step(s + 1 < S ? s + 1 : s);
    if (end) load_a(i0 + s / nt);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int kk = 0; kk + 1 < KK; ++kk) {
      const int c = kk & 1;
      zl_frag(cur, kk + 1, f[c ^ 1], wm0, wn0, lane);
      zl_step(f[c], acc);
      zl_interleave();
    }
    __builtin_amdgcn_sched_barrier(0);
    cf.stage(nxt);
    __syncthreads();
    zl_frag(nxt, 0, f[0], wm0, wn0, lane);
    zl_step(f[(KK - 1) & 1], acc);
    zl_interleave();
    if (end) flush();
  };
  if (S > 0) {
    fetch_step(0);
    cf.stage(buf0);
  }
  __syncthreads();
  if (S > 0) zl_frag(buf0, 0, f[0], wm0, wn0, lane);
  // two steps per pass (S is even), so both LDS stages are addressed statically
  for (int s = 0; s < S; s += 2) {
    tile(s, buf0, buf1);
    tile(s + 1, buf1, buf0);
  }

  float* out = reinterpret_cast<float*>(part + (long)split * nmu * nmu);
#pragma unroll
  for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < ZL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + fm * 16 + Mfma<float>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        if (row < col) continue;
        const float val = (row == col && pp == 1) ? 0.f : (float)acc64[fm][fn][v];   // Hermitian: real diagonal
        out[((long)row * nmu + col) * 2 + pp] = val;
        if (row > col) out[((long)col * nmu + row) * 2 + pp] = pp ? -val : val;
      }
}

}  // namespace

bool core32_fits(int nmu, int nc) { return nmu >= ZL::BM && nmu % ZL::BM == 0 && nc >= 32 && nc % 32 == 0; }

// Split of the occupied index: the count s (at most max_split) that minimises the
// makespan rounds(s) * ceil(nv / s), with rounds(s) the rounds of one workgroup per
// CU that tiles * s workgroups take; the smallest such s (fewest partial sums).
int core32_splits(int nmu, int nv, int max_split) {
  const int nti = nmu / ZL::BM, tiles = nti * (nti + 1);
  const long slots = cu_count();
  int best = 1;
  long best_cost = -1;
  for (int s = 1; s <= std::max(1, std::min(nv, max_split)); ++s) {
    const long rounds = ((long)tiles * s + slots - 1) / slots;
    const long cost = rounds * ((nv + s - 1) / s);
    if (best_cost < 0 || cost < best_cost) { best_cost = cost; best = s; }
  }
  return best;
}

hipError_t core32_partial(int nmu, int nv, int nc, const void* pm, const double* w, void* part, int nsplit,
                          hipStream_t st, int batch) {
  if (!core32_fits(nmu, nc) || nsplit < 1 || nsplit > nv) return hipErrorInvalidValue;
  const int nti = nmu / ZL::BM, total = nti * (nti + 1);
  const unsigned gx = 8u * (unsigned)((total + 7) / 8);
  hipLaunchKernelGGL(core32_kernel, dim3(gx, nsplit, batch), dim3(ZL::NT), 0, st, nmu, nv, nc, (const z64*)pm, w,
                     (c32*)part, nsplit, total);
  return hipGetLastError();
}

}  // namespace isdf
