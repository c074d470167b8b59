// Single-precision complex GEMMs with both operands k-major, on the engine of
// kmajor.h: the two output products of the SMW step in the mixed path,
//   W^T = alpha T^T X^T            (plain: complex64 out)
//   eps~^{-1} = I + alpha W X^H    (Hermitian: lower tiles only, complex128 out,
//                                   upper triangle mirrored, real diagonal)
//   X^H X                          (the Coulomb Gram, Hermitian with no identity,
//                                   from a [plane wave][point] copy of X)
// with X^T and W^T stored [point][plane wave].  One workgroup per CU walks its
// XCD's contiguous share of the tiles (no inter-workgroup synchronisation) and
// prefetches the next tile's first K tile under the current epilogue.  Only
// full tiles are handled here (M % 128 = N % 64 = K % 16 = 0); the caller keeps
// the general GEMM for anything else.
//
// Tail split: when a share does not fill whole rounds, its leftover tiles are
// cut along K so that every workgroup of the XCD takes one slice (given scratch
// for the slices); gemm32_tail_kernel then adds the slices in a fixed order and
// applies the epilogue, so the last round is as full as the others.
#include "internal.h"
#include "kmajor.h"

#include <algorithm>
#include <cmath>

namespace isdf {

// lower-triangle tile list of a square (nti 128-row) x (2 nti 64-column) grid,
// row-major: row bm holds the tiles bn <= 2 bm + 1, so rows [0, bm) hold bm (bm + 1)
__device__ __forceinline__ void herm_tile(int id, int& bm, int& bn) {
  int r = (int)((sqrtf(4.f * (float)id + 1.f) - 1.f) * 0.5f);
  while (r * (r + 1) > id) --r;
  while ((r + 1) * (r + 2) <= id) ++r;
  bm = r;
  bn = id - r * (r + 1);
}

// Full rounds and split tail of one XCD's share of `total` tiles (nper workgroups
// per XCD, nt K tiles): tiles [lo, lo + nfull) run whole, the ntail after them are
// cut into `split` K slices each (split = 1: no tail).
struct TailPlan {
  int lo, nfull, ntail, split;
};
__host__ __device__ inline TailPlan tail_plan(int xcd, int total, int nper, int nt, bool allow) {
  const int per = (total + 7) / 8;
  const int lo = xcd * per, hi = total < lo + per ? total : lo + per;
  const int cnt = hi > lo ? hi - lo : 0;
  TailPlan t{lo, cnt, 0, 1};
  if (!allow || nper < 2) return t;
  const int rounds = cnt / nper, rest = cnt - rounds * nper;
  if (rest == 0) return t;
  int sp = nper / rest;
  if (sp > nt) sp = nt;
  if (sp < 2) return t;
  t.nfull = rounds * nper;
  t.ntail = rest;
  t.split = sp;
  return t;
}

template <bool HERM>
__device__ __forceinline__ void tile_origin(int id, int ntj, int& m0, int& n0) {
  int bm, bn;
  if (HERM) herm_tile(id, bm, bn);
  else { bm = id / ntj; bn = id % ntj; }
  m0 = bm * ZL::BM;
  n0 = bn * ZL::BN;
}

// EVEN (plain output, an even number of K tiles): the first K tile is staged before
// the tile loop and each tile's last K tile stages the next tile's first one, so no
// tile starts with a wait on global loads (which the memory counter would retire
// only after the previous tile's output stores).  The Hermitian output goes through
// the LDS, so it stages at the start of every tile.
template <bool HERM, bool EVEN>
__global__ __launch_bounds__(ZL::NT) __attribute__((amdgpu_waves_per_eu(2)))
void gemm32_kernel(int ntj, int total, int K, const c32* A, long lda, float sa, const c32* B, long ldb,
                   float sb, void* C, long ldc, float alpha, float diag, float* tail_ws) {
  __shared__ float smem[2 * (ZL::AS + ZL::BS)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % ZL::WGM) * ZL::WTM, wn0 = (wave / ZL::WGM) * ZL::WTN;
  const int xcd = blockIdx.x % 8, nper = gridDim.x / 8, j = blockIdx.x / 8;
  const int nt = K / ZL::BK;
  const TailPlan tp = tail_plan(xcd, total, nper, nt, tail_ws != nullptr);
  const int lo = tp.lo, hi = tp.lo + tp.nfull;
  ZFetch zf;
  ZFrag frag[2];
  zf.init(tid, lda, ldb);
  static_assert(!(HERM && EVEN), "the Hermitian epilogue uses the LDS stages");
  if (lo + j < hi) {
    int m0, n0;
    tile_origin<HERM>(lo + j, ntj, m0, n0);
    zf.fetch(A, lda, B, ldb, m0, n0, 0);
    if (EVEN) {
      zf.stage(smem, sa, sb);
      __syncthreads();
      zl_frag(smem, 0, frag[0], wm0, wn0, lane);
    }
  }
  const int rc = lane & 15, part = rc & 1;
  for (int id = lo + j; id < hi; id += nper) {
    int m0, n0, nm0 = 0, nn0 = 0;
    tile_origin<HERM>(id, ntj, m0, n0);
    const bool has_next = id + nper < hi;
    if (has_next) tile_origin<HERM>(id + nper, ntj, nm0, nn0);
    f4 acc[ZL::FM][ZL::FN];
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn) acc[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
    zl_range(smem, zf, frag, 0, nt, EVEN, sa, sb, A, lda, B, ldb, m0, n0, has_next, nm0, nn0, 0, acc, wm0,
             wn0, lane);
    if (!HERM) {
#pragma unroll
      for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
        for (int fn = 0; fn < ZL::FN; ++fn)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = m0 + wm0 + fm * 16 + Mfma<float>::row(lane, v);
            const int c = n0 + wn0 + fn * 8 + (rc >> 1);
            reinterpret_cast<float*>(C)[((long)r * ldc + c) * 2 + part] = alpha * acc[fm][fn][v];
          }
      continue;
    }
    // Hermitian output through LDS (free after the K loop's last barrier): the tile
    // [128 rows][64 complex, stride 65] is written once row by row (lower part) and
    // once column by column as the conjugate mirror, both as contiguous rows of the
    // complex128 output.
    float* ts = smem;
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = wm0 + fm * 16 + Mfma<float>::row(lane, v);
          const int c = wn0 + fn * 8 + (rc >> 1);
          ts[(r * 65 + c) * 2 + part] = alpha * acc[fm][fn][v];
        }
    __syncthreads();
    double* o = reinterpret_cast<double*>(C);
    for (int e = tid; e < ZL::BM * ZL::BN; e += ZL::NT) {   // lower part, row-major
      const int r = e / ZL::BN, c = e % ZL::BN, gr = m0 + r, gc = n0 + c;
      if (gr < gc) continue;
      const float re = ts[(r * 65 + c) * 2], im = ts[(r * 65 + c) * 2 + 1];
      *reinterpret_cast<double2*>(o + ((long)gr * ldc + gc) * 2) =
          gr == gc ? double2{(double)diag + (double)re, 0.0} : double2{(double)re, (double)im};
    }
    for (int e = tid; e < ZL::BM * ZL::BN; e += ZL::NT) {   // mirror: output row gc, contiguous along gr
      const int c = e / ZL::BM, r = e % ZL::BM, gr = m0 + r, gc = n0 + c;
      if (gr <= gc) continue;
      const float re = ts[(r * 65 + c) * 2], im = ts[(r * 65 + c) * 2 + 1];
      *reinterpret_cast<double2*>(o + ((long)gc * ldc + gr) * 2) = double2{(double)re, -(double)im};
    }
    __syncthreads();   // the next tile stages into the same LDS
  }
  // one K slice of a leftover tile: raw partial sum to the scratch, [row][column] complex64
  if (tp.ntail > 0 && j < tp.ntail * tp.split) {
    const int tt = j / tp.split, ks = j % tp.split;
    int m0, n0;
    tile_origin<HERM>(hi + tt, ntj, m0, n0);
    const int t0 = ks * nt / tp.split, t1 = (ks + 1) * nt / tp.split;
    const c32* As = A + (long)t0 * ZL::BK * lda;
    const c32* Bs = B + (long)t0 * ZL::BK * ldb;
    f4 acc[ZL::FM][ZL::FN];
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn) acc[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
    zf.fetch(As, lda, Bs, ldb, m0, n0, 0);
    zl_range(smem, zf, frag, 0, t1 - t0, false, sa, sb, As, lda, Bs, ldb, m0, n0, false, 0, 0, 0, acc, wm0,
             wn0, lane);
    float* ws = tail_ws + (size_t)(xcd * nper + j) * ZL::BM * ZL::BN * 2;
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = wm0 + fm * 16 + Mfma<float>::row(lane, v);
          const int c = wn0 + fn * 8 + (rc >> 1);
          ws[(r * ZL::BN + c) * 2 + part] = acc[fm][fn][v];
        }
  }
}

// Leftover tiles of the split tail: workgroup (xcd, t, chunk) adds, for 512 complex
// elements of that XCD's tail tile t (two per thread, one 16-byte load per slice),
// the K slices in slice order, scales by alpha and writes them as the main
// kernel's epilogue would.
constexpr int TAIL_CHUNKS = ZL::BM * ZL::BN / 512;

template <bool HERM>
__global__ __launch_bounds__(256) void gemm32_tail_kernel(int ntj, int total, int nper, int nt, const float* tail_ws,
                                                          void* C, long ldc, float alpha, float diag) {
  const int xcd = blockIdx.x, t = blockIdx.y;
  const TailPlan tp = tail_plan(xcd, total, nper, nt, true);
  if (t >= tp.ntail) return;
  int m0, n0;
  tile_origin<HERM>(tp.lo + tp.nfull + t, ntj, m0, n0);
  const size_t unit = (size_t)ZL::BM * ZL::BN * 2;
  const float* ws = tail_ws + (size_t)(xcd * nper + t * tp.split) * unit;
  const int e = 2 * (blockIdx.z * 256 + threadIdx.x);   // elements e, e + 1 (same row)
  f4 acc = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int ks = 0; ks < tp.split; ++ks) acc += *reinterpret_cast<const f4*>(ws + ks * unit + 2 * e);
  acc *= alpha;
  const int r = e / ZL::BN, c = e % ZL::BN, gr = m0 + r;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int gc = n0 + c + h;
    const float re = acc[2 * h], im = acc[2 * h + 1];
    if (!HERM) {
      reinterpret_cast<float2*>(C)[(long)gr * ldc + gc] = float2{re, im};
      continue;
    }
    double* o = reinterpret_cast<double*>(C);
    if (gr < gc) continue;
    *reinterpret_cast<double2*>(o + ((long)gr * ldc + gc) * 2) =
        gr == gc ? double2{(double)diag + (double)re, 0.0} : double2{(double)re, (double)im};
    if (gr > gc) *reinterpret_cast<double2*>(o + ((long)gc * ldc + gr) * 2) = double2{(double)re, -(double)im};
  }
}

// dst[c][r] = src[r * lds + c] for r < rows, c < cols (complex64), through 32 x 32 LDS tiles
__global__ __launch_bounds__(256) void transpose_c32_kernel(int rows, int cols, const c32* __restrict__ src, long lds,
                                                            c32* __restrict__ dst) {
  __shared__ c32 t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    if (r < rows && c < cols) t[k][tx] = src[(long)r * lds + c];
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) dst[(long)c * rows + r] = t[tx][k];
  }
}

hipError_t transpose_c32(int rows, int cols, const void* src, long lds, void* dst, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(transpose_c32_kernel, dim3(cdiv(cols, 32), cdiv(rows, 32)), dim3(256), 0, st, rows, cols,
                     (const c32*)src, lds, (c32*)dst);
  return hipGetLastError();
}

size_t gemm32_tail_bytes(int wg_per_cu) {
  const int wpc = std::max(1, std::min(wg_per_cu, 4));
  const int g = 8 * ((wpc * cu_count() + 7) / 8);
  return (size_t)g * ZL::BM * ZL::BN * 2 * sizeof(float);
}

bool gemm32_fits(int M, int N, int K, const void* A, long lda, const void* B, long ldb) {
  const bool aligned = (lda & 1) == 0 && (ldb & 1) == 0 &&
                       ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0;
  return aligned && M > 0 && N > 0 && K > 0 && M % ZL::BM == 0 && N % ZL::BN == 0 && K % ZL::BK == 0;
}

hipError_t gemm32_kmajor(int M, int N, int K, const void* A, long lda, bool conjA, const void* B, long ldb,
                         bool conjB, void* C, long ldc, bool herm_identity, double alpha, hipStream_t st,
                         int wg_per_cu, void* tail_ws, size_t tail_bytes, double diag) {
  if (!gemm32_fits(M, N, K, A, lda, B, ldb) || (herm_identity && M != N)) return hipErrorNotSupported;
  const int nti = M / ZL::BM, ntj = N / ZL::BN;
  const int total = herm_identity ? nti * (nti + 1) : nti * ntj;
  if (total == 0) return hipSuccess;
  const int wpc = std::max(1, std::min(wg_per_cu, 4));
  const int gfull = 8 * ((wpc * cu_count() + 7) / 8);
  // fewer tiles than workgroups: one round, its tiles cut along K over the whole grid
  // when the scratch holds every slice (a long-K product such as the Coulomb Gram);
  // otherwise one workgroup per tile
  const bool cut_all = total < gfull && tail_ws && tail_bytes >= (size_t)gfull * ZL::BM * ZL::BN * 2 * sizeof(float);
  const int g = cut_all ? gfull : std::max(8, std::min(gfull, 8 * (int)cdiv(total, 8)));
  const float sa = conjA ? -1.f : 1.f, sb = conjB ? -1.f : 1.f;
  const int nper = g / 8, nt = K / ZL::BK;
  // the split tail only with scratch for every workgroup's slice
  const size_t need = (size_t)g * ZL::BM * ZL::BN * 2 * sizeof(float);
  float* ws = (tail_ws && tail_bytes >= need) ? (float*)tail_ws : nullptr;
  bool any_tail = false;
  for (int x = 0; ws && x < 8; ++x) any_tail |= tail_plan(x, total, nper, nt, true).ntail > 0;
  if (!any_tail) ws = nullptr;
  if (herm_identity)
    hipLaunchKernelGGL((gemm32_kernel<true, false>), dim3(g), dim3(ZL::NT), 0, st, ntj, total, K, (const c32*)A,
                       lda, sa, (const c32*)B, ldb, sb, C, ldc, (float)alpha, (float)diag, ws);
  else if (nt % 2 == 0)
    hipLaunchKernelGGL((gemm32_kernel<false, true>), dim3(g), dim3(ZL::NT), 0, st, ntj, total, K, (const c32*)A,
                       lda, sa, (const c32*)B, ldb, sb, C, ldc, (float)alpha, (float)diag, ws);
  else
    hipLaunchKernelGGL((gemm32_kernel<false, false>), dim3(g), dim3(ZL::NT), 0, st, ntj, total, K, (const c32*)A,
                       lda, sa, (const c32*)B, ldb, sb, C, ldc, (float)alpha, (float)diag, ws);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !ws) return e;
  int max_tail = 0;
  for (int x = 0; x < 8; ++x) max_tail = std::max(max_tail, tail_plan(x, total, nper, nt, true).ntail);
  const dim3 tg(8, max_tail, TAIL_CHUNKS);
  if (herm_identity)
    hipLaunchKernelGGL(gemm32_tail_kernel<true>, tg, dim3(256), 0, st, ntj, total, nper, nt, ws, C, ldc, (float)alpha,
                       (float)diag);
  else
    hipLaunchKernelGGL(gemm32_tail_kernel<false>, tg, dim3(256), 0, st, ntj, total, nper, nt, ws, C, ldc,
                       (float)alpha, (float)diag);
  return hipGetLastError();
}

}  // namespace isdf
