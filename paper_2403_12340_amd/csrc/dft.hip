// Grid-side kernels: orbitals at the interpolation points, pair weights, the
// Coulomb factor, and the unitary 3-D DFT of the N_mu real-space columns
// sampled on the plane-wave list.
//
// The DFT is pruned to the frequencies the plane-wave list needs: with the
// sphere of NG vectors spanning kx of the n0 x-frequencies, the transform runs
//   x:  T1[y][a]   = sum_x Z[z][y][x] twx[a][x]          (kx of n0 outputs)
//   y:  T2[z][d]   = sum_y T1[y][a_d] twy[b_d][y]         (only (x, y) pairs in use)
//   z:  ZG[g]      = sum_z T2[z][d_g] twz[c_g][z]          (only listed vectors)
// Stages x and y run in one kernel per (point, z-plane) slab held in LDS
// (one coalesced read of the slab); stage z reads the small T2.  Each
// twiddle table carries its 1/sqrt(n) so the product is unitary.
#include "internal.h"

#include <algorithm>
#include "tile.h"

#include <cmath>

namespace isdf {

__global__ void widen_kernel(const double* src, z64* dst, long count) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = z64{src[i], 0.0};
}

hipError_t widen_real(const double* src, void* dst, long count, hipStream_t st) {
  hipLaunchKernelGGL(widen_kernel, dim3(cdiv(count, 256)), dim3(256), 0, st, src, (z64*)dst, count);
  return hipGetLastError();
}

// pm[n][mu] = psi[n * nr + mu_idx[mu]]
__global__ void gather_kernel(const z64* psi, long nr, int ns, const int* mu, int nmu, z64* pm) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  const int n = blockIdx.y;
  if (m < nmu && n < ns) pm[(long)n * nmu + m] = psi[(long)n * nr + mu[m]];
}

hipError_t gather_points(const void* psi, long nr, int ns, const int* mu, int nmu, void* pm,
                         hipStream_t st) {
  hipLaunchKernelGGL(gather_kernel, dim3(cdiv(nmu, 256), ns), dim3(256), 0, st, (const z64*)psi, nr,
                     ns, mu, nmu, (z64*)pm);
  return hipGetLastError();
}

// w[i][j] = D / (D^2 + omega^2), D = e_i - e_{nv + j}
__global__ void weights_kernel(const double* e, int nv, int nc, double omega, double* w) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nv * nc) return;
  const int i = (int)(idx / nc), j = (int)(idx % nc);
  const double d = e[i] - e[nv + j];
  w[idx] = d / (d * d + omega * omega);
}

hipError_t pair_weights(const double* e, int nv, int nc, double omega, double* w, hipStream_t st) {
  hipLaunchKernelGGL(weights_kernel, dim3(cdiv((long)nv * nc, 256)), dim3(256), 0, st, e, nv, nc, omega, w);
  return hipGetLastError();
}

// Device-side gap check for energies that never reach the host: sets `bit` in
// *status unless every energy is finite and max(occupied) < min(empty).
// One workgroup; a fixed-shape tree reduction in LDS.
__global__ __launch_bounds__(256) void gap_kernel(const double* e, int nv, int nc, int* status, int bit) {
  __shared__ double vmax[256], cmin[256];
  __shared__ int nonfinite[256];
  const int t = threadIdx.x;
  double a = -INFINITY, b = INFINITY;
  int bad = 0;
  for (int i = t; i < nv + nc; i += 256) {
    const double x = e[i];
    bad |= !isfinite(x);
    if (i < nv) a = fmax(a, x);
    else b = fmin(b, x);
  }
  vmax[t] = a; cmin[t] = b; nonfinite[t] = bad;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (t < s) {
      vmax[t] = fmax(vmax[t], vmax[t + s]);
      cmin[t] = fmin(cmin[t], cmin[t + s]);
      nonfinite[t] |= nonfinite[t + s];
    }
    __syncthreads();
  }
  if (t == 0 && (nonfinite[0] || !(vmax[0] < cmin[0]))) atomicOr(status, bit);
}

hipError_t check_gap(const double* e, int nv, int nc, int* status, int bit, hipStream_t st) {
  hipLaunchKernelGGL(gap_kernel, dim3(1), dim3(256), 0, st, e, nv, nc, status, bit);
  return hipGetLastError();
}

// sqrt(V(G)) = sqrt(v_scale 4 pi / |G|^2), 0 at G = 0; G = sum_d m_d b_d, b_d rows of recip (2 pi included)
__global__ void coulomb_kernel(const int* miller, int ng, const double* recip, double v_scale,
                               double* sqrtv) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const double m0 = miller[3 * g], m1 = miller[3 * g + 1], m2 = miller[3 * g + 2];
  double g2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double gc = m0 * recip[c] + m1 * recip[3 + c] + m2 * recip[6 + c];
    g2 += gc * gc;
  }
  sqrtv[g] = (g2 > 0.0) ? sqrt(v_scale * 4.0 * M_PI / g2) : 0.0;
}

hipError_t coulomb_sqrt(const int* miller, int ng, const double* recip, double v_scale, double* sqrtv,
                        hipStream_t st) {
  hipLaunchKernelGGL(coulomb_kernel, dim3(cdiv(ng, 256)), dim3(256), 0, st, miller, ng, recip, v_scale, sqrtv);
  return hipGetLastError();
}

// tw[a][x] = exp(-2 pi i m_a x / n) / sqrt(n), phase reduced exactly mod n first
template <typename T>
__global__ void twiddle_kernel(const int* mlist, int nm, int n, cx<T>* tw) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nm * n) return;
  const int a = idx / n, x = idx % n;
  long ph = ((long)mlist[a] * x) % n;
  if (ph < 0) ph += n;
  double s, c;
  sincospi(-2.0 * (double)ph / (double)n, &s, &c);
  const double sc = 1.0 / sqrt((double)n);
  tw[idx] = cx<T>{(T)(c * sc), (T)(s * sc)};
}

hipError_t dft_twiddles(const int* mlist, int nm, int n, bool f32, void* tw, hipStream_t st) {
  if (f32) hipLaunchKernelGGL((twiddle_kernel<float>), dim3(cdiv(nm * n, 256)), dim3(256), 0, st, mlist, nm, n, (c32*)tw);
  else hipLaunchKernelGGL((twiddle_kernel<double>), dim3(cdiv(nm * n, 256)), dim3(256), 0, st, mlist, nm, n, (z64*)tw);
  return hipGetLastError();
}

__host__ __device__ inline int up16(int n) { return (n + 15) / 16 * 16; }

// One workgroup walks `zb` consecutive z-planes (slabs) of one point.  Per slab
// (n1 x n0: y rows, x contiguous):
//   x stage  T1^T (a x y) = TWX (a x x) . slab^T (x x y)    MFMA, 2 x 2 waves
//   y stage  T2   (a x b) = T1^T (a x y) . TWY^T (y x b)    MFMA, 2 x 2 waves
// and only the (a, b) pairs of the plane-wave list are stored, z-contiguous:
// t2[mu][d][z].  a and b run in chunks of 32.  The slab is copied into LDS as
// it lies in memory ([y][x], read as an n-major B operand); T1 overwrites it as
// [y][a] (the k-major A operand of the y stage); the twiddle chunks [x][a] and
// [y][b] stay resident across slabs, the next slab is prefetched into registers
// under the MFMAs, and each lane's pair indices are looked up once.  Every LDS
// value outside the live ranges is finite (zeroed once, then only data) and the
// twiddle padding is zero, so padded rows and columns contribute exactly zero.
template <typename T>
using TileXS = Tile<T, 32, 64, 16, 2, 2>;  // x stage: M a (32), N y (64), K x
template <typename T>
using TileYS = Tile<T, 32, 32, 16, 2, 2>;  // y stage: M a (32), N b (32), K y; LDA = LDB = 33

constexpr int XY_NT = 256;
constexpr int XY_LDS = 65;                 // slab row stride (complex): n-major B operand of the x stage

template <typename T>
static size_t xy_lds_bytes() {
  return sizeof(cx<T>) * (64 * XY_LDS + 2 * 64 * 33);
}

// PF = slab elements per thread held in registers (n0 n1 <= 256 PF)
template <typename T, int PF>
__global__ __launch_bounds__(XY_NT) void dft_xy_kernel(DftPlan p, const cx<T>* __restrict__ zt,
                                                       cx<T>* __restrict__ t2, int zb) {
  typedef TileXS<T> TX;
  typedef TileYS<T> TY;
  static_assert(TX::LDA == 33 && TY::LDA == 33 && TY::LDB == 33, "chunk strides");
  extern __shared__ unsigned char lds_raw[];
  cx<T>* Ss = reinterpret_cast<cx<T>*>(lds_raw);   // slab [y][x] (stride 65), then T1 [y][a] (stride 33)
  cx<T>* Xs = Ss + 64 * XY_LDS;                     // TWX^T chunk [x][a]: A operand of the x stage
  cx<T>* Ys = Xs + 64 * 33;                         // TWY^T chunk [y][b]: B operand of the y stage
  const int nzb = (p.n2 + zb - 1) / zb;
  const int mu = blockIdx.x / nzb, z0 = (blockIdx.x % nzb) * zb, z1 = min(p.n2, z0 + zb);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int x16 = up16(p.n0), y16 = up16(p.n1);
  const int nslab = p.n0 * p.n1;
  const bool one_chunk = p.kx <= 32 && p.ky <= 32;
  const cx<T>* twx = reinterpret_cast<const cx<T>*>(p.twx);
  const cx<T>* twy = reinterpret_cast<const cx<T>*>(p.twy);
  for (int i = tid; i < 64 * XY_LDS; i += XY_NT) Ss[i] = cx<T>{(T)0, (T)0};
  auto load_chunk = [&](cx<T>* dst, const cx<T>* tw, int nk, int kpad, int nlist, int c0) {
    // dst[k][c] = tw[(c0 + c) * nk + k] for k < nk and c0 + c < nlist, else 0
    for (int i = tid; i < kpad * 32; i += XY_NT) {
      const int k = i / 32, c = i % 32;
      const bool ok = k < nk && c0 + c < nlist;
      const cx<T> v = tw[ok ? (c0 + c) * nk + k : 0];
      dst[k * 33 + c] = cx<T>{ok ? v.re : (T)0, ok ? v.im : (T)0};  // component selects stay in registers
    }
  };
  const int wm0 = (wave % 2) * 16, xn0 = (wave / 2) * TX::WTN, yn0 = (wave / 2) * TY::WTN;
  const int rc = lane & 15, part = rc & 1;
  // this lane's y-stage outputs (a, b) -> pair index, for the single-chunk case
  int dl[TY::FN][4];
#pragma unroll
  for (int fn = 0; fn < TY::FN; ++fn)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int a = wm0 + Mfma<T>::row(lane, v), b = yn0 + fn * 8 + (rc >> 1);
      dl[fn][v] = (one_chunk && a < p.kx && b < p.ky) ? p.dmap[a * p.ky + b] : -1;
    }
  T pfr[PF], pfi[PF];  // slab prefetch (split re / im keeps it in registers)
  if (z0 < z1) {
    const cx<T>* src = zt + ((long)mu * p.n2 + z0) * nslab;
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int i = tid + e * XY_NT;
      const cx<T> v = src[i < nslab ? i : 0];
      pfr[e] = v.re; pfi[e] = v.im;
    }
  }
  T* ssr = reinterpret_cast<T*>(Ss);
  for (int z = z0; z < z1; ++z) {
    __syncthreads();  // previous slab's y stage is done with Ss
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int i = tid + e * XY_NT;
      if (i < nslab) Ss[(i / p.n0) * XY_LDS + i % p.n0] = cx<T>{pfr[e], pfi[e]};
    }
    if (z + 1 < z1) {  // next slab into registers, under this slab's MFMAs
      const cx<T>* src = zt + ((long)mu * p.n2 + z + 1) * nslab;
#pragma unroll
      for (int e = 0; e < PF; ++e) {
        const int i = tid + e * XY_NT;
        const cx<T> v = src[i < nslab ? i : 0];
        pfr[e] = v.re; pfi[e] = v.im;
      }
    }
    for (int a0 = 0; a0 < p.kx; a0 += 32) {
      if (z == z0 || !one_chunk) load_chunk(Xs, twx, p.n0, x16, p.kx, a0);
      __syncthreads();
      // x stage for rows a in [a0, a0 + 32): acc = TWX . slab^T (rows a, columns y)
      typename TX::acc_t acc[TX::FM][TX::FN];
      zero_acc<TX>(acc);
      for (int kc = 0; kc < x16; kc += 16) tile_mma_bn<T, TX>(Xs + kc * 33, Ss + kc, XY_LDS, acc, wm0, xn0, lane);
      __syncthreads();  // every wave is done reading the slab
#pragma unroll
      for (int fn = 0; fn < TX::FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = wm0 + Mfma<T>::row(lane, v);
          const int y = xn0 + fn * 8 + (rc >> 1);
          ssr[(y * 33 + a) * 2 + part] = acc[0][fn][v];  // T1[y][a]
        }
      for (int b0 = 0; b0 < p.ky; b0 += 32) {
        if (z == z0 || !one_chunk) load_chunk(Ys, twy, p.n1, y16, p.ky, b0);
        __syncthreads();
        typename TY::acc_t acc2[TY::FM][TY::FN];
        zero_acc<TY>(acc2);
        for (int kc = 0; kc < y16; kc += 16) tile_mma<T, TY>(Ss + kc * 33, Ys + kc * 33, acc2, wm0, yn0, lane);
        T* t2r = reinterpret_cast<T*>(t2);
#pragma unroll
        for (int fn = 0; fn < TY::FN; ++fn)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            int d = dl[fn][v];
            if (!one_chunk) {
              const int a = a0 + wm0 + Mfma<T>::row(lane, v), b = b0 + yn0 + fn * 8 + (rc >> 1);
              d = (a < p.kx && b < p.ky) ? p.dmap[a * p.ky + b] : -1;
            }
            if (d >= 0) t2r[(((long)mu * p.nd + d) * p.n2 + z) * 2 + part] = acc2[0][fn][v];
          }
        if (b0 + 32 < p.ky) __syncthreads();  // Ys is reloaded for the next chunk
      }
      if (a0 + 32 < p.kx) {
        __syncthreads();  // T1 chunk consumed: restore the slab for the next row chunk
        for (int i = tid; i < nslab; i += XY_NT) Ss[(i / p.n0) * XY_LDS + i % p.n0] = zt[((long)mu * p.n2 + z) * nslab + i];
      }
    }
  }
}

bool dft_supported(int n0, int n1, int n2, int kx, int ky, Prec compute) {
  (void)kx; (void)ky;  // any list length: the x and y stages run in chunks of 32 frequencies
  if (n1 > 64 || n0 > 64) return false;  // one 64 x 64 slab per MFMA tile
  if (n2 > 64) return false;             // one z-line per wave in the z stage
  const size_t bytes = compute == P64 ? xy_lds_bytes<double>() : xy_lds_bytes<float>();
  return bytes <= 160 * 1024;
}

template <typename T, int PF>
static void xy_launch(const DftPlan& p, const void* zt, void* t2, int zb, dim3 grid, hipStream_t st) {
  const size_t lds = xy_lds_bytes<T>();
  static bool attr_set[64] = {};  // once per device, outside any later stream capture
  int dev = 0;
  (void)hipGetDevice(&dev);
  if (dev < 0 || dev >= 64 || !attr_set[dev]) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dft_xy_kernel<T, PF>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (dev >= 0 && dev < 64) attr_set[dev] = true;
  }
  hipLaunchKernelGGL((dft_xy_kernel<T, PF>), grid, dim3(XY_NT), lds, st, p, (const cx<T>*)zt, (cx<T>*)t2, zb);
}

template <typename T>
static void xy_dispatch(const DftPlan& p, const void* zt, void* t2, int zb, dim3 grid, hipStream_t st) {
  const int nslab = p.n0 * p.n1;
  if (nslab <= 4 * XY_NT) xy_launch<T, 4>(p, zt, t2, zb, grid, st);
  else if (nslab <= 9 * XY_NT) xy_launch<T, 9>(p, zt, t2, zb, grid, st);
  else xy_launch<T, 16>(p, zt, t2, zb, grid, st);
}

hipError_t dft_xy(Prec compute, const DftPlan& p, const void* zt, void* t2, hipStream_t st) {
  if (p.n0 > 64 || p.n1 > 64) return hipErrorInvalidValue;
  const int zb = std::max(1, std::min(p.n2, p.zb));
  const int nzb = (p.n2 + zb - 1) / zb;
  const dim3 grid((unsigned)(p.nmu * nzb));
  if (compute == P64) xy_dispatch<double>(p, zt, t2, zb, grid, st);
  else xy_dispatch<float>(p, zt, t2, zb, grid, st);
  return hipGetLastError();
}

// z stage: zg[mu][g] = scale[g] sum_z t2[mu][d_g][z] twz[c_g][z], one thread per
// (plane wave, point).  Threads take the plane waves in (x, y)-pair order, so the
// ~NG/nd neighbours that share a pair read the same z-line (few distinct cache
// lines per load); each thread runs four independent partial sums.
template <typename T>
__global__ __launch_bounds__(256) void dft_z_kernel(DftPlan p, const cx<T>* __restrict__ t2, cx<T>* __restrict__ zg,
                                                    const double* __restrict__ scale) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  if (e >= p.ng) return;
  const int g = p.gd_list[e];
  const int d = p.g_d[g], c = p.g_cz[g];
  const cx<T>* twz = reinterpret_cast<const cx<T>*>(p.twz) + (long)c * p.n2;
  const cx<T>* line = t2 + ((long)mu * p.nd + d) * p.n2;
  T sr[4] = {0, 0, 0, 0}, si[4] = {0, 0, 0, 0};
  int z = 0;
  for (; z + 4 <= p.n2; z += 4) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const cx<T> v = line[z + u], w = twz[z + u];
      sr[u] += v.re * w.re - v.im * w.im;
      si[u] += v.re * w.im + v.im * w.re;
    }
  }
  for (; z < p.n2; ++z) {
    const cx<T> v = line[z], w = twz[z];
    sr[0] += v.re * w.re - v.im * w.im;
    si[0] += v.re * w.im + v.im * w.re;
  }
  const T sc = scale ? (T)scale[g] : (T)1;
  zg[(long)mu * p.ng + g] = cx<T>{((sr[0] + sr[1]) + (sr[2] + sr[3])) * sc, ((si[0] + si[1]) + (si[2] + si[3])) * sc};
}

hipError_t dft_z(Prec compute, const DftPlan& p, const void* t2, void* zg, const double* scale,
                 hipStream_t st) {
  const dim3 grid(cdiv(p.ng, 256), p.nmu);
  if (compute == P64)
    hipLaunchKernelGGL((dft_z_kernel<double>), grid, dim3(256), 0, st, p, (const z64*)t2, (z64*)zg, scale);
  else
    hipLaunchKernelGGL((dft_z_kernel<float>), grid, dim3(256), 0, st, p, (const c32*)t2, (c32*)zg, scale);
  return hipGetLastError();
}

}  // namespace isdf
