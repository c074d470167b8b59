// Single-precision complex GEMMs with both operands k-major, on the engine of
// kmajor.h: the two output products of the SMW step in the mixed path,
//   W^T = alpha T^T X^T            (plain: complex64 out)
//   eps~^{-1} = I + alpha W X^H    (Hermitian: lower tiles only, complex128 out,
//                                   upper triangle mirrored, real diagonal)
// with X^T and W^T stored [point][plane wave].  One workgroup per CU walks its
// XCD's contiguous share of the tiles (no inter-workgroup synchronisation) and
// prefetches the next tile's first K tile under the current epilogue.  Only
// full tiles are handled here (M % 128 = N % 64 = K % 16 = 0); the caller keeps
// the general GEMM for anything else.
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

template <bool HERM>
__global__ __launch_bounds__(ZL::NT) __attribute__((amdgpu_waves_per_eu(3)))
void gemm32_kernel(int ntj, int total, int K, const c32* A, long lda, float sa, const c32* B, long ldb,
                   float sb, void* C, long ldc, float alpha) {
  __shared__ float smem[2 * (ZL::AS + ZL::BS)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % ZL::WGM) * ZL::WTM, wn0 = (wave / ZL::WGM) * ZL::WTN;
  const int xcd = blockIdx.x % 8, nper = gridDim.x / 8, j = blockIdx.x / 8;
  const int per = (total + 7) / 8;
  const int lo = xcd * per, hi = min(total, lo + per);
  const int nt = K / ZL::BK;
  auto origin = [&](int id, int& m0, int& n0) {
    int bm, bn;
    if (HERM) herm_tile(id, bm, bn);
    else { bm = id / ntj; bn = id % ntj; }
    m0 = bm * ZL::BM;
    n0 = bn * ZL::BN;
  };
  ZFetch zf;
  zf.init(tid, lda, ldb);
  if (lo + j < hi) {
    int m0, n0;
    origin(lo + j, m0, n0);
    zf.fetch(A, lda, B, ldb, m0, n0, 0);
  }
  const int rc = lane & 15, part = rc & 1;
  for (int id = lo + j; id < hi; id += nper) {
    int m0, n0, nm0 = 0, nn0 = 0;
    origin(id, m0, n0);
    const bool has_next = id + nper < hi;
    if (has_next) origin(id + nper, nm0, nn0);
    f4 acc[ZL::FM][ZL::FN];
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn) acc[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
    zl_loop_full(smem, zf, nt, nt, sa, sb, A, lda, B, ldb, m0, n0, has_next, nm0, nn0, acc, acc, wm0, wn0, lane);
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
          gr == gc ? double2{1.0 + (double)re, 0.0} : double2{(double)re, (double)im};
    }
    for (int e = tid; e < ZL::BM * ZL::BN; e += ZL::NT) {   // mirror: output row gc, contiguous along gr
      const int c = e / ZL::BM, r = e % ZL::BM, gr = m0 + r, gc = n0 + c;
      if (gr <= gc) continue;
      const float re = ts[(r * 65 + c) * 2], im = ts[(r * 65 + c) * 2 + 1];
      *reinterpret_cast<double2*>(o + ((long)gc * ldc + gr) * 2) = double2{(double)re, -(double)im};
    }
    __syncthreads();   // the next tile stages into the same LDS
  }
}

bool gemm32_fits(int M, int N, int K, const void* A, long lda, const void* B, long ldb) {
  const bool aligned = (lda & 1) == 0 && (ldb & 1) == 0 &&
                       ((reinterpret_cast<uintptr_t>(A) | reinterpret_cast<uintptr_t>(B)) & 15) == 0;
  return aligned && M > 0 && N > 0 && K > 0 && M % ZL::BM == 0 && N % ZL::BN == 0 && K % ZL::BK == 0;
}

hipError_t gemm32_kmajor(int M, int N, int K, const void* A, long lda, bool conjA, const void* B, long ldb,
                         bool conjB, void* C, long ldc, bool herm_identity, double alpha, hipStream_t st,
                         int wg_per_cu) {
  if (!gemm32_fits(M, N, K, A, lda, B, ldb) || (herm_identity && M != N)) return hipErrorNotSupported;
  const int nti = M / ZL::BM, ntj = N / ZL::BN;
  const int total = herm_identity ? nti * (nti + 1) : nti * ntj;
  if (total == 0) return hipSuccess;
  const int wpc = std::max(1, std::min(wg_per_cu, 4));
  const int g = std::max(8, std::min(8 * ((wpc * cu_count() + 7) / 8), 8 * (int)cdiv(total, 8)));
  const float sa = conjA ? -1.f : 1.f, sb = conjB ? -1.f : 1.f;
  if (herm_identity)
    hipLaunchKernelGGL(gemm32_kernel<true>, dim3(g), dim3(ZL::NT), 0, st, ntj, total, K, (const c32*)A, lda, sa,
                       (const c32*)B, ldb, sb, C, ldc, (float)alpha);
  else
    hipLaunchKernelGGL(gemm32_kernel<false>, dim3(g), dim3(ZL::NT), 0, st, ntj, total, K, (const c32*)A, lda, sa,
                       (const c32*)B, ldb, sb, C, ldc, (float)alpha);
  return hipGetLastError();
}

}  // namespace isdf
