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
#include "kmajor.h"   // cu_count
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

// Fused x, y and z stages for lists with at most 32 x- and y-frequencies (the
// plane-wave spheres of the Coulomb Gram).  A workgroup of ceil(kx / 8) waves
// walks an equal run of consecutive (point, z-plane) slabs; wave w owns the
// x-frequencies [8 w, 8 w + 8).  Per slab (n1 x n0, y rows, x contiguous):
//   x stage  T1 (y x a_w)  = slab (y x x) . TWX^T (x x a_w)     rows y in 16s
//   y stage  T2 (b x a_w)  = TWY (b x y) . T1 (y x a_w)         rows b in 16s
// T1 goes through a region of LDS private to the wave (no workgroup barrier
// between the stages), and T2 overwrites it in place.  After one barrier every
// thread adds T2[b_g][a_g] twz[c_g][z] into the running sums of its plane waves
// (ng / blockDim of them, in registers), so T2 never reaches HBM.  The sums of
// each point's run go to `part` [mu][piece][g], and dft_zsum_kernel adds the
// pieces and applies the scale.  Padding rows and columns of the slab are zero (set
// once); twiddle padding is zero, so padded terms contribute exactly zero.
// Register budgets (slab elements and plane waves per thread) of the two
// instantiations: up to 48^3-like shapes, and up to 64^3-like ones (FP32 only).
constexpr int FUSED_PF_S = 12, FUSED_GPT_S = 24, FUSED_PF_L = 16, FUSED_GPT_L = 32;

// g workgroups; workgroup w transforms the slabs [w S / g, (w + 1) S / g) of the
// S = nmu n2 slabs in (point, z) order, so the work is balanced whatever nmu and
// the number of resident workgroups are.  The run of one point inside a
// workgroup's range is one piece of that point's z sum (at most pmax pieces).
struct FusedShape {
  int nw, nt, fmx, fmb, pf, gpt, x2, y2, ls, la, wsz, g, pmax;
  size_t lds;
};

// last workgroup whose range starts at or before slab x
__host__ __device__ inline int fused_owner(long x, long S, int g) {
  const long w = ((x + 1) * g - 1) / S;
  return (int)(w < g - 1 ? w : g - 1);
}

template <typename T>
static bool fused_shape(const DftPlan& p, FusedShape& f) {
  if (p.kx < 1 || p.kx > 32 || p.ky < 1 || p.ky > 32 || p.kz < 1 || p.kz > 64) return false;
  if (p.n0 > 64 || p.n1 > 64 || p.n2 > 64) return false;
  f.nw = (p.kx + 7) / 8;
  f.nt = 64 * f.nw;
  f.fmx = (p.n1 + 15) / 16;
  f.fmb = (p.ky + 15) / 16;
  f.pf = (p.n0 * p.n1 + f.nt - 1) / f.nt;
  f.gpt = (p.ng + f.nt - 1) / f.nt;
  const bool large_ok = sizeof(T) == 4;
  if (f.pf > (large_ok ? FUSED_PF_L : FUSED_PF_S) || f.gpt > (large_ok ? FUSED_GPT_L : FUSED_GPT_S)) return false;
  f.x2 = (p.n0 + 3) & ~3;   // K extents in whole pairs of MFMA steps (zero padding)
  f.y2 = (p.n1 + 3) & ~3;
  f.ls = f.x2 + 1;
  f.la = 8 * f.nw + 1;
  f.wsz = std::max(16 * f.fmx, 32) * 9;
  const size_t el = (size_t)16 * f.fmx * f.ls + (size_t)f.x2 * f.la + (size_t)f.y2 * 33 + (size_t)f.nw * f.wsz +
                    (size_t)p.n2 * p.kz;
  f.g = f.pmax = 0;   // set by the launcher
  f.lds = el * sizeof(cx<T>);
  return f.lds <= 160 * 1024;
}

// issue order of one MFMA step: the next step's LDS reads (N + 1 of them) between
// this step's N MFMAs
template <int N>
__device__ __forceinline__ void fused_interleave() {
#pragma unroll
  for (int r = 0; r < N; ++r) {
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // DS read
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // MFMA
  }
  __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
}

template <typename T, int PF, int GPT, int FMX>
__global__ __launch_bounds__(256) void dft_fused_kernel(DftPlan p, FusedShape f, const cx<T>* __restrict__ zt,
                                                        cx<T>* __restrict__ out, const double* __restrict__ scale) {
  static_assert(GPT % 8 == 0, "plane waves are summed in groups of 8");
  constexpr int FMB = 2;   // b rows in two blocks of 16 (ky <= 32; zero twiddle columns beyond ky)
  extern __shared__ unsigned char lds_raw[];
  const int rows = 16 * FMX;
  cx<T>* Ss = reinterpret_cast<cx<T>*>(lds_raw);   // slab [y][x], rows x ls
  cx<T>* Xs = Ss + rows * f.ls;                     // TWX^T [x][a], x2 x la
  cx<T>* Ys = Xs + f.x2 * f.la;                     // TWY^T [y][b], y2 x 33
  cx<T>* Tw = Ys + f.y2 * 33;                       // per wave: T1 [y][a_w], then T2 [b][a_w]; stride 9
  cx<T>* Zs = Tw + f.nw * f.wsz;                    // twz [z][c]
  const int nt = f.nt, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long S = (long)p.nmu * p.n2;
  const long s0 = (long)blockIdx.x * S / f.g, s1 = (long)(blockIdx.x + 1) * S / f.g;
  const int nslab = p.n0 * p.n1;
  const cx<T>* twx = reinterpret_cast<const cx<T>*>(p.twx);
  const cx<T>* twy = reinterpret_cast<const cx<T>*>(p.twy);
  const cx<T>* twz = reinterpret_cast<const cx<T>*>(p.twz);
  const cx<T> zero{(T)0, (T)0};
  for (int i = tid; i < rows * f.ls; i += nt) Ss[i] = zero;
  for (int i = tid; i < f.x2 * f.la; i += nt) {
    const int k = i / f.la, c = i % f.la;
    Xs[i] = (k < p.n0 && c < p.kx) ? twx[c * p.n0 + k] : zero;
  }
  for (int i = tid; i < f.y2 * 33; i += nt) {
    const int k = i / 33, c = i % 33;
    Ys[i] = (k < p.n1 && c < p.ky) ? twy[c * p.n1 + k] : zero;
  }
  for (int i = tid; i < p.n2 * p.kz; i += nt) {
    const int z = i / p.kz, c = i % p.kz;
    Zs[i] = twz[c * p.n2 + z];
  }
  // this thread's plane waves g = tid + nt j: T2 offset in Tw | z-frequency << 16;
  // slots past the list hold code 0 (summed like the rest, never stored)
  uint32_t gcode[GPT];
  cx<T> zacc[GPT];
#pragma unroll
  for (int j = 0; j < GPT; ++j) {
    const int g = tid + nt * j;
    zacc[j] = zero;
    gcode[j] = 0;
    if (g < p.ng) {
      const int d = p.g_d[g], a = p.d_ax[d];
      gcode[j] = (uint32_t)((a >> 3) * f.wsz + p.d_by[d] * 9 + (a & 7)) | ((uint32_t)p.g_cz[g] << 16);
    }
  }
  // slab element e of this thread: i = tid + nt e at Ss[(i / n0) ls + i % n0], stepped incrementally
  const int r0 = tid / p.n0, c0 = tid % p.n0, dr = nt / p.n0, dc = nt % p.n0;
  T pfr[PF], pfi[PF];
  int mu = 0;   // point of the current run
  auto fetch = [&](int z) {
    const char* src = reinterpret_cast<const char*>(zt + ((long)mu * p.n2 + z) * nslab);
#pragma unroll
    for (int e = 0; e < PF; ++e) {
      const int i = tid + nt * e;
      const cx<T> v = *reinterpret_cast<const cx<T>*>(src + (uint32_t)(i < nslab ? i : 0) * (uint32_t)sizeof(cx<T>));
      pfr[e] = v.re; pfi[e] = v.im;
    }
  };
  __syncthreads();  // Ss zeroed before any slab element lands
  const int i16 = lane & 15, q = lane >> 4, rc = lane & 15, part = rc & 1;
  const int bpart = ((q & 1) == (i16 & 1)) ? 0 : 1;
  const T bsign = ((q & 1) == 1 && (i16 & 1) == 0) ? (T)-1 : (T)1;
  const T* SsR = reinterpret_cast<const T*>(Ss);
  const T* XsR = reinterpret_cast<const T*>(Xs);
  const T* YsR = reinterpret_cast<const T*>(Ys);
  T* TwR = reinterpret_cast<T*>(Tw + wave * f.wsz);
  for (long sb = s0; sb < s1;) {   // runs of one point
  mu = (int)(sb / p.n2);
  const int z0 = (int)(sb % p.n2), z1 = (int)min((long)p.n2, z0 + (s1 - sb));
#pragma unroll
  for (int j = 0; j < GPT; ++j) zacc[j] = zero;
  fetch(z0);
  for (int z = z0; z < z1; ++z) {
    {
      int r = r0, c = c0;
#pragma unroll
      for (int e = 0; e < PF; ++e) {
        if (tid + nt * e < nslab) Ss[r * f.ls + c] = cx<T>{pfr[e], pfi[e]};
        r += dr; c += dc;
        if (c >= p.n0) { c -= p.n0; ++r; }
      }
    }
    if (z + 1 < z1) fetch(z + 1);  // next slab in flight under this slab's MFMAs
    __syncthreads();
    // x stage: rows y (fmx blocks of 16), columns a in [8 wave, 8 wave + 8), k = x
    typename Mfma<T>::acc_t acc1[FMX];
#pragma unroll
    for (int fm = 0; fm < FMX; ++fm)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc1[fm][v] = 0;
    {
      // fragments of step kk + 1 are read while the MFMAs of step kk issue; the
      // step index is clamped, so the read past the end is an in-bounds repeat
      const int nk = f.x2 / 2, sa = 4, sb = 4 * f.la;
      const T* ap = SsR + (i16 * f.ls + (q >> 1)) * 2 + (q & 1);
      const T* bp = XsR + ((q >> 1) * f.la + 8 * wave + (i16 >> 1)) * 2 + bpart;
      T a0[FMX], a1[FMX], b0, b1;
      auto rd = [&](int kk, T (&a)[FMX], T& b) {
        kk = min(kk, nk - 1);
#pragma unroll
        for (int fm = 0; fm < FMX; ++fm) a[fm] = ap[fm * 32 * f.ls + kk * sa];
        b = bsign * bp[kk * sb];
      };
      rd(0, a0, b0);
      for (int kk = 0; kk < nk; kk += 2) {   // nk is even
        rd(kk + 1, a1, b1);
#pragma unroll
        for (int fm = 0; fm < FMX; ++fm) acc1[fm] = Mfma<T>::op(a0[fm], b0, acc1[fm]);
        fused_interleave<FMX>();
        rd(kk + 2, a0, b0);
#pragma unroll
        for (int fm = 0; fm < FMX; ++fm) acc1[fm] = Mfma<T>::op(a1[fm], b1, acc1[fm]);
        fused_interleave<FMX>();
      }
    }
#pragma unroll
    for (int fm = 0; fm < FMX; ++fm)
#pragma unroll
      for (int v = 0; v < 4; ++v) TwR[((16 * fm + Mfma<T>::row(lane, v)) * 9 + (rc >> 1)) * 2 + part] = acc1[fm][v];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // y stage: rows b (fmb blocks of 16), columns a of this wave, k = y
    typename Mfma<T>::acc_t acc2[FMB];
#pragma unroll
    for (int fb = 0; fb < FMB; ++fb)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc2[fb][v] = 0;
    {
      const int nk = f.y2 / 2;
      const T* ap = YsR + ((q >> 1) * 33 + i16) * 2 + (q & 1);
      const T* bp = TwR + ((q >> 1) * 9 + (i16 >> 1)) * 2 + bpart;
      T a0[FMB], a1[FMB], b0, b1;
      auto rd = [&](int kk, T (&a)[FMB], T& b) {
        kk = min(kk, nk - 1);
#pragma unroll
        for (int fb = 0; fb < FMB; ++fb) a[fb] = ap[fb * 32 + kk * 4 * 33];
        b = bsign * bp[kk * 4 * 9];
      };
      rd(0, a0, b0);
      for (int kk = 0; kk < nk; kk += 2) {   // nk is even
        rd(kk + 1, a1, b1);
#pragma unroll
        for (int fb = 0; fb < FMB; ++fb) acc2[fb] = Mfma<T>::op(a0[fb], b0, acc2[fb]);
        fused_interleave<FMB>();
        rd(kk + 2, a0, b0);
#pragma unroll
        for (int fb = 0; fb < FMB; ++fb) acc2[fb] = Mfma<T>::op(a1[fb], b1, acc2[fb]);
        fused_interleave<FMB>();
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();   // every lane has read T1 before T2 overwrites it
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
    for (int fb = 0; fb < FMB; ++fb)
#pragma unroll
      for (int v = 0; v < 4; ++v) TwR[((16 * fb + Mfma<T>::row(lane, v)) * 9 + (rc >> 1)) * 2 + part] = acc2[fb][v];
    __syncthreads();
    // z stage: running sums of this thread's plane waves
    const cx<T>* zrow = Zs + z * p.kz;
#pragma unroll
    for (int j0 = 0; j0 < GPT; j0 += 8) {
      __builtin_amdgcn_sched_barrier(0);   // bounds the LDS reads in flight (register pressure)
#pragma unroll
      for (int j = j0; j < j0 + 8; ++j) {
        // opaque to the optimiser: decoded per use, not hoisted out of the slab loop as
        // two more registers per plane wave
        uint32_t code = gcode[j];
        asm volatile("" : "+v"(code));
        const cx<T> v = Tw[code & 0xffffu], w = zrow[code >> 16];
        zacc[j].re += v.re * w.re - v.im * w.im;
        zacc[j].im += v.re * w.im + v.im * w.re;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < GPT; ++j) {   // this run is piece (workgroup - first owner) of the point's sum
    if (tid + nt * j >= p.ng) continue;
    const int g = tid + nt * j;
    const int piece = (int)blockIdx.x - fused_owner((long)mu * p.n2, S, f.g);
    out[((long)mu * f.pmax + piece) * p.ng + g] = zacc[j];
  }
  sb += z1 - z0;
  }
}

// Warp-specialised fused pass (FP32, grids with n0 and n1 rounding to the same 2 NK):
// a workgroup has two groups of nw MFMA waves and PIPE_ZW z-waves.  At step t group k
// runs the x and y stages of slab s0 + 2 t + k (its twiddle fragments held in
// registers) from the slab buffers of parity t, while the z-waves store the pair of
// step t + 1 (loaded during step t - 1) into the buffers of the other parity, issue the
// loads of the pair of step t + 2, and add the T2 of both slabs of step t - 1 into the
// running plane-wave sums (slab order; a point's run ends with the store of its piece).
// One barrier per step: the pair of step t staged and T2 of step t - 1 complete.  Slabs
// and T2 are double buffered by step parity; T1 stays in a region private to each MFMA
// wave.  The sums, the pieces and the twiddle padding follow dft_fused_kernel.
// Roles of the z-waves: wave w runs on SIMD w % 4, and a z-wave on a SIMD that hosts
// more MFMA waves than the others gets few issue cycles until those MFMA waves are done
// (measured: its step's work ends about 3000 cycles after theirs).  Every z-wave stages
// an equal share of the slabs; when the MFMA waves are spread unevenly only the z-waves
// on the other SIMDs sum plane waves, otherwise every z-wave does.
constexpr int PIPE_ZW = 6;   // z-waves per workgroup
// register budgets of a z-wave: slab elements per thread and slab, plane waves per
// summing thread
constexpr int PIPE_PF = 6, PIPE_GPT = 16;
struct PipeShape {
  int nw, nt, ls, ssz, wsz, t2sz, g, pmax;
  unsigned sum_mask;   // summing z-waves (bit zi of wave 2 nw + zi)
  size_t lds;
};

// summing z-waves for nw MFMA waves per group (see above)
static unsigned pipe_roles(int nw) {
  int m[4] = {0, 0, 0, 0};
  for (int w = 0; w < 2 * nw; ++w) ++m[w & 3];
  const int mx = std::max(std::max(m[0], m[1]), std::max(m[2], m[3]));
  const int mn = std::min(std::min(m[0], m[1]), std::min(m[2], m[3]));
  unsigned mask = 0;
  for (int zi = 0; zi < PIPE_ZW; ++zi)
    if (mx == mn || m[(2 * nw + zi) & 3] < mx) mask |= 1u << zi;
  return mask;
}

// One z-wave of the warp-specialised pass: it stages slabs (PFX elements per slab and
// thread, thread st0 of nst), and with GPTX > 0 it sums plane waves (GPTX per thread,
// thread zt0 of nzt).  Every z-wave passes the same barriers as the MFMA waves.
template <int PFX, int GPTX>
__device__ __forceinline__ void pipe_zwave(const DftPlan& p, const PipeShape& f, const c32* __restrict__ zt,
                                           c32* __restrict__ out, c32* Ss, const c32* T2, const c32* Zs,
                                           uint32_t* Gc, int s0, int s1, int nsteps, int nslab, int S, int st0,
                                           int nst, int zt0, int nzt) {
  const c32 zero{0.f, 0.f};
  // this thread's plane waves g = zt0 + nzt j: T2 offset | z-frequency << 16, kept in LDS
  // (read by this thread only); slots past the list hold code 0 (summed, never stored)
  c32 zacc[GPTX > 0 ? GPTX : 1];
#pragma unroll
  for (int j = 0; j < GPTX; ++j) zacc[j] = zero;
  if constexpr (GPTX > 0) {
    // two rounds of independent loads (the pairs and z-frequencies of all the thread's
    // plane waves, then the pairs' x and y indices) instead of a dependent chain per
    // plane wave
    int dj[GPTX], cz[GPTX];
#pragma unroll
    for (int j = 0; j < GPTX; ++j) {
      const int g = zt0 + nzt * j;
      dj[j] = g < p.ng ? p.g_d[g] : -1;
      cz[j] = g < p.ng ? p.g_cz[g] : 0;
    }
#pragma unroll
    for (int j = 0; j < GPTX; ++j) {
      uint32_t code = 0;
      if (dj[j] >= 0) {
        const int a = p.d_ax[dj[j]];
        code = (uint32_t)((a >> 3) * 288 + p.d_by[dj[j]] * 9 + (a & 7)) | ((uint32_t)cz[j] << 16);
      }
      Gc[j * nzt + zt0] = code;
    }
  }
  const int r0 = st0 / p.n0, c0 = st0 % p.n0, dr = nst / p.n0, dc = nst % p.n0;
  float pfr[2][PFX > 0 ? PFX : 1], pfi[2][PFX > 0 ? PFX : 1];
  // the pair of step t into registers (slabs past the range are not read)
  auto fetch = [&](int t) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int sl = s0 + 2 * t + k;
      if (sl >= s1) continue;
      const char* src = reinterpret_cast<const char*>(zt + (long)sl * nslab);
#pragma unroll
      for (int e = 0; e < PFX; ++e) {
        const int i = st0 + nst * e;
        const c32 v = *reinterpret_cast<const c32*>(src + (uint32_t)(i < nslab ? i : 0) * (uint32_t)sizeof(c32));
        pfr[k][e] = v.re; pfi[k][e] = v.im;
      }
    }
  };
  auto store = [&](int t) {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (s0 + 2 * t + k >= s1) continue;
      c32* dst = Ss + ((t & 1) * 2 + k) * f.ssz;
      int r = r0, c = c0;
#pragma unroll
      for (int e = 0; e < PFX; ++e) {
        if (st0 + nst * e < nslab) dst[r * f.ls + c] = c32{pfr[k][e], pfi[k][e]};
        r += dr; c += dc;
        if (c >= p.n0) { c -= p.n0; ++r; }
      }
    }
  };
  if constexpr (PFX > 0) {
    fetch(0);
    store(0);
    if (1 < nsteps) fetch(1);
  }
  for (int t = 0; t <= nsteps; ++t) {
    __syncthreads();   // the pair of step t staged; T2 of step t - 1 complete
    // the pair of step t + 1 (loaded during the previous step) into the other buffers,
    // whose last reader was step t - 1; then the loads of the pair of step t + 2
    if constexpr (PFX > 0) {
      if (t + 1 < nsteps) store(t + 1);
      if (t + 2 < nsteps) fetch(t + 2);
    }
    if (GPTX > 0 && t > 0) {
#pragma unroll 1
      for (int k = 0; k < 2; ++k) {
        const int sp = s0 + 2 * (t - 1) + k;   // slab summed now
        if (sp >= s1) break;
        const c32* t2 = T2 + (((t - 1) & 1) * 2 + k) * f.t2sz;
        const c32* zrow = Zs + (sp % p.n2) * p.kz;
#pragma unroll
        for (int j0 = 0; j0 < GPTX; j0 += 2) {
          __builtin_amdgcn_sched_barrier(0);   // bounds the LDS reads in flight (register pressure)
#pragma unroll
          for (int j = j0; j < j0 + 2 && j < GPTX; ++j) {
            const uint32_t code = Gc[j * nzt + zt0];
            const c32 v = t2[code & 0xffffu], wz = zrow[code >> 16];
            zacc[j].re += v.re * wz.re - v.im * wz.im;
            zacc[j].im += v.re * wz.im + v.im * wz.re;
          }
        }
        if (sp + 1 == s1 || (sp + 1) % p.n2 == 0) {   // the run of this point ends: store its piece
          const int mu = sp / p.n2;
          const int piece = (int)blockIdx.x - fused_owner((long)mu * p.n2, S, f.g);
          c32* ob = out + ((long)mu * f.pmax + piece) * p.ng;
          // one running index, opaque to the optimiser: no per-plane-wave index is
          // hoisted out of the slab loop into a register of its own
          int g = zt0;
          asm volatile("" : "+v"(g));
#pragma unroll
          for (int j = 0; j < GPTX; ++j) {
            if (g < p.ng) ob[g] = zacc[j];
            zacc[j] = zero;
            g += nzt;
          }
        }
      }
    }
  }
}

template <int FMX, int NK, int GPT, int PF>
__global__ __launch_bounds__(768) __attribute__((amdgpu_waves_per_eu(3))) void dft_pipe_kernel(DftPlan p, PipeShape f, const c32* __restrict__ zt,
                                                       c32* __restrict__ out) {
  constexpr int FMB = 2;   // b rows in two blocks of 16 (ky <= 32)
  extern __shared__ unsigned char lds_raw[];
  c32* Ss = reinterpret_cast<c32*>(lds_raw);   // four slabs [parity][k][y][x], ssz each (rows x ls)
  c32* Tw = Ss + 4 * f.ssz;                     // per MFMA wave: T1 [y][a_w], stride 9
  c32* T2 = Tw + 2 * f.nw * f.wsz;              // [parity][k][nw][32][9]: T2 [b][a_w]
  c32* Zs = T2 + 4 * f.t2sz;                    // twz [z][c]
  uint32_t* Gc = reinterpret_cast<uint32_t*>(Zs + p.n2 * p.kz);   // plane-wave codes [j][z-thread]
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool zw = wave >= 2 * f.nw;
  const int S = p.nmu * p.n2;   // slabs (the launcher keeps this in int range)
  const int s0 = (int)((long)blockIdx.x * S / f.g), s1 = (int)((long)(blockIdx.x + 1) * S / f.g);
  const int nsteps = (s1 - s0 + 1) / 2;
  const int nslab = p.n0 * p.n1;
  const c32* twx = reinterpret_cast<const c32*>(p.twx);
  const c32* twy = reinterpret_cast<const c32*>(p.twy);
  const c32* twz = reinterpret_cast<const c32*>(p.twz);
  const c32 zero{0.f, 0.f};
  for (int i = tid; i < 4 * f.ssz; i += f.nt) Ss[i] = zero;
  for (int i = tid; i < p.n2 * p.kz; i += f.nt) {
    const int z = i / p.kz, c = i % p.kz;
    Zs[i] = twz[c * p.n2 + z];
  }
  if (s0 >= s1) return;   // the whole workgroup
  __syncthreads();        // the zeroed slabs and the z twiddles before any use
  const int i16 = lane & 15, q = lane >> 4, rc = lane & 15, part = rc & 1;
  if (!zw) {
    // ---- MFMA waves: group k = wave / nw, x-frequency block w = wave % nw
    const int k = wave / f.nw, w = wave % f.nw;
    const int bpart = ((q & 1) == (i16 & 1)) ? 0 : 1;
    const float bsign = ((q & 1) == 1 && (i16 & 1) == 0) ? -1.f : 1.f;
    float xb[NK], ya[NK][FMB];   // x-stage B and y-stage A fragments (zero padded)
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      const int kx = (q >> 1) + 2 * kk, c = 8 * w + (i16 >> 1);
      const c32 v = (kx < p.n0 && c < p.kx) ? twx[c * p.n0 + kx] : zero;
      xb[kk] = bsign * (bpart ? v.im : v.re);
#pragma unroll
      for (int fb = 0; fb < FMB; ++fb) {
        const int cy = i16 + 16 * fb;
        const c32 u = (kx < p.n1 && cy < p.ky) ? twy[cy * p.n1 + kx] : zero;
        ya[kk][fb] = (q & 1) ? u.im : u.re;
      }
    }
    float* TwR = reinterpret_cast<float*>(Tw + wave * f.wsz);
    for (int t = 0; t <= nsteps; ++t) {
      const bool mine = t < nsteps && s0 + 2 * t + k < s1;
      __syncthreads();   // the pair of step t staged; T2 of step t - 1 read by the z-waves
      Mfma<float>::acc_t acc1[FMX];
      if (mine) {
#pragma unroll
        for (int fm = 0; fm < FMX; ++fm) acc1[fm] = f4{0.f, 0.f, 0.f, 0.f};
        const float* SsR = reinterpret_cast<const float*>(Ss + ((t & 1) * 2 + k) * f.ssz);
        const float* ap = SsR + (i16 * f.ls + (q >> 1)) * 2 + (q & 1);
        float a0[FMX], a1[FMX];
#pragma unroll
        for (int fm = 0; fm < FMX; ++fm) a0[fm] = ap[fm * 32 * f.ls];
#pragma unroll
        for (int kk = 0; kk < NK; kk += 2) {
#pragma unroll
          for (int fm = 0; fm < FMX; ++fm) a1[fm] = ap[fm * 32 * f.ls + (kk + 1) * 4];
#pragma unroll
          for (int fm = 0; fm < FMX; ++fm) acc1[fm] = Mfma<float>::op(a0[fm], xb[kk], acc1[fm]);
          fused_interleave<FMX>();
          if (kk + 2 < NK) {
#pragma unroll
            for (int fm = 0; fm < FMX; ++fm) a0[fm] = ap[fm * 32 * f.ls + (kk + 2) * 4];
          }
#pragma unroll
          for (int fm = 0; fm < FMX; ++fm) acc1[fm] = Mfma<float>::op(a1[fm], xb[kk + 1], acc1[fm]);
          fused_interleave<FMX>();
        }
#pragma unroll
        for (int fm = 0; fm < FMX; ++fm)
#pragma unroll
          for (int v = 0; v < 4; ++v) TwR[((16 * fm + Mfma<float>::row(lane, v)) * 9 + (rc >> 1)) * 2 + part] = acc1[fm][v];
        // T1 is private to this wave: its writes before its reads
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        Mfma<float>::acc_t acc2[FMB];
#pragma unroll
        for (int fb = 0; fb < FMB; ++fb) acc2[fb] = f4{0.f, 0.f, 0.f, 0.f};
        const float* bp = TwR + ((q >> 1) * 9 + (i16 >> 1)) * 2 + bpart;
        float b0 = bsign * bp[0], b1;
#pragma unroll
        for (int kk = 0; kk < NK; kk += 2) {
          b1 = bsign * bp[(kk + 1) * 4 * 9];
#pragma unroll
          for (int fb = 0; fb < FMB; ++fb) acc2[fb] = Mfma<float>::op(ya[kk][fb], b0, acc2[fb]);
          if (kk + 2 < NK) b0 = bsign * bp[(kk + 2) * 4 * 9];
#pragma unroll
          for (int fb = 0; fb < FMB; ++fb) acc2[fb] = Mfma<float>::op(ya[kk + 1][fb], b1, acc2[fb]);
        }
        float* T2R = reinterpret_cast<float*>(T2 + ((t & 1) * 2 + k) * f.t2sz + w * 288);
#pragma unroll
        for (int fb = 0; fb < FMB; ++fb)
#pragma unroll
          for (int v = 0; v < 4; ++v) T2R[((16 * fb + Mfma<float>::row(lane, v)) * 9 + (rc >> 1)) * 2 + part] = acc2[fb][v];
      }
    }
  } else {
    // ---- z-waves: the zi-th; its index among all z-threads (staging) and among the summing ones
    const int zi = wave - 2 * f.nw;
    const int st0 = 64 * zi + lane, nst = 64 * PIPE_ZW;
    const int zt0 = 64 * __builtin_popcount(f.sum_mask & ((1u << zi) - 1u)) + lane,
              nzt = 64 * __builtin_popcount(f.sum_mask);
    if ((f.sum_mask >> zi) & 1u)
      pipe_zwave<PF, GPT>(p, f, zt, out, Ss, T2, Zs, Gc, s0, s1, nsteps, nslab, S, st0, nst, zt0, nzt);
    else
      pipe_zwave<PF, 0>(p, f, zt, out, Ss, T2, Zs, Gc, s0, s1, nsteps, nslab, S, st0, nst, zt0, nzt);
  }
}

// zg[mu][g] = scale[g] sum_j part[mu][j][g] over the point's pieces, in piece order
template <typename T>
__global__ void dft_zsum_kernel(const cx<T>* __restrict__ part, int pmax, long S, int g_wg, int n2, int nmu, int ng,
                                const double* __restrict__ scale, cx<T>* __restrict__ zg) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x, mu = blockIdx.y;
  if (g >= ng) return;
  const int np = fused_owner((long)(mu + 1) * n2 - 1, S, g_wg) - fused_owner((long)mu * n2, S, g_wg) + 1;
  T re = 0, im = 0;
  for (int j = 0; j < np; ++j) {
    const cx<T> v = part[((long)mu * pmax + j) * ng + g];
    re += v.re;
    im += v.im;
  }
  const T sc = scale ? (T)scale[g] : (T)1;
  zg[(long)mu * ng + g] = cx<T>{re * sc, im * sc};
}

template <typename T, int PF, int GPT, int FMX>
static hipError_t fused_kernel_launch(const DftPlan& p, FusedShape& f, const void* zt, void* part,
                                      size_t part_bytes, hipStream_t st) {
  const void* fn = reinterpret_cast<const void*>(&dft_fused_kernel<T, PF, GPT, FMX>);
  // per device: the LDS attribute once (outside any later stream capture), and the
  // resident workgroups per CU for the last shape asked
  static bool attr_set[64] = {};
  static int occ_lds[64] = {}, occ_nt[64] = {}, occ[64] = {};
  int dev = 0;
  (void)hipGetDevice(&dev);
  const bool cache = dev >= 0 && dev < 64;
  if (!cache || !attr_set[dev]) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (cache) attr_set[dev] = true;
  }
  int per_cu = 0;
  if (cache && occ_lds[dev] == (int)f.lds && occ_nt[dev] == f.nt) {
    per_cu = occ[dev];
  } else {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, f.nt, f.lds) != hipSuccess || per_cu < 1) per_cu = 1;
    if (cache) { occ_lds[dev] = (int)f.lds; occ_nt[dev] = f.nt; occ[dev] = per_cu; }
  }
  // one resident round of workgroups (at least 4 slabs each); fewer if the pieces
  // per point would overflow the scratch
  const long S = (long)p.nmu * p.n2;
  long g = std::min<long>((long)per_cu * cu_count(), std::max<long>(1, S / 4));
  for (;;) {
    int pmax = 1;
    for (int mu = 0; mu < p.nmu; ++mu)
      pmax = std::max(pmax, fused_owner((long)(mu + 1) * p.n2 - 1, S, (int)g) - fused_owner((long)mu * p.n2, S, (int)g) + 1);
    f.g = (int)g;
    f.pmax = pmax;
    if ((size_t)p.nmu * pmax * p.ng * sizeof(cx<T>) <= part_bytes) break;
    if (g == 1) return hipErrorNotSupported;
    g = std::max<long>(1, g * 3 / 4);
  }
  hipLaunchKernelGGL((dft_fused_kernel<T, PF, GPT, FMX>), dim3((unsigned)f.g), dim3(f.nt), f.lds, st, p, f,
                     (const cx<T>*)zt, (cx<T>*)part, nullptr);
  return hipGetLastError();
}



// even NK (K steps of both stages) and the register budgets of its instantiation
static bool pipe_shape(const DftPlan& p, PipeShape& f, int& nk) {
  const int x2 = (p.n0 + 3) & ~3, y2 = (p.n1 + 3) & ~3;
  if (x2 != y2 || x2 > 48) return false;   // larger slabs need more registers than a wave has
  if (p.kx < 1 || p.kx > 24 || p.ky < 1 || p.ky > 32 || p.kz < 1 || p.kz > 64 || p.n2 > 64) return false;
  if ((long)p.nmu * p.n2 > 0x7fffffffL) return false;
  nk = x2 / 2;
  f.nw = (p.kx + 7) / 8;
  f.nt = 128 * f.nw + 64 * PIPE_ZW;
  f.sum_mask = pipe_roles(f.nw);
  const int fmx = (2 * nk + 15) / 16, nzt = 64 * __builtin_popcount(f.sum_mask);
  const long gpt = cdiv(p.ng, nzt), pf = cdiv((long)p.n0 * p.n1, 64 * PIPE_ZW);
  if (gpt > PIPE_GPT || pf > PIPE_PF) return false;
  f.ls = x2 + 1;
  f.ssz = 16 * fmx * f.ls;
  f.wsz = 16 * fmx * 9;
  f.t2sz = f.nw * 288;
  f.g = f.pmax = 0;
  f.lds = ((size_t)4 * f.ssz + (size_t)2 * f.nw * f.wsz + 4 * (size_t)f.t2sz + (size_t)p.n2 * p.kz) * sizeof(c32) +
          (size_t)PIPE_GPT * nzt * sizeof(uint32_t);
  return f.lds <= 160 * 1024;
}

template <int NK>
static hipError_t pipe_kernel_launch(const DftPlan& p, PipeShape& f, const void* zt, void* part, size_t part_bytes,
                                     hipStream_t st) {
  constexpr int FMX = (2 * NK + 15) / 16, GPT = PIPE_GPT, PF = PIPE_PF;
  const void* fn = reinterpret_cast<const void*>(&dft_pipe_kernel<FMX, NK, GPT, PF>);
  static bool attr_set[64] = {};
  int dev = 0;
  (void)hipGetDevice(&dev);
  const bool cache = dev >= 0 && dev < 64;
  if (!cache || !attr_set[dev]) {
    (void)hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (cache) attr_set[dev] = true;
  }
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, f.nt, f.lds) != hipSuccess || per_cu < 1) per_cu = 1;
  // one resident round of workgroups (at least 4 slabs each); fewer if the pieces
  // per point would overflow the scratch
  const long S = (long)p.nmu * p.n2;
  long g = std::min<long>((long)per_cu * cu_count(), std::max<long>(1, S / 4));
  for (;;) {
    int pmax = 1;
    for (int mu = 0; mu < p.nmu; ++mu)
      pmax = std::max(pmax, fused_owner((long)(mu + 1) * p.n2 - 1, S, (int)g) - fused_owner((long)mu * p.n2, S, (int)g) + 1);
    f.g = (int)g;
    f.pmax = pmax;
    if ((size_t)p.nmu * pmax * p.ng * sizeof(c32) <= part_bytes) break;
    if (g == 1) return hipErrorNotSupported;
    g = std::max<long>(1, g * 3 / 4);
  }
  hipLaunchKernelGGL((dft_pipe_kernel<FMX, NK, GPT, PF>), dim3((unsigned)f.g), dim3(f.nt), f.lds, st, p, f,
                     (const c32*)zt, (c32*)part);
  return hipGetLastError();
}

// hipErrorNotSupported when no instantiation covers the shape
static hipError_t pipe_launch(const DftPlan& p, PipeShape& f, const void* zt, void* part, size_t part_bytes,
                              hipStream_t st) {
  int nk = 0;
  if (!pipe_shape(p, f, nk)) return hipErrorNotSupported;
  switch (nk) {
    case 4: return pipe_kernel_launch<4>(p, f, zt, part, part_bytes, st);
    case 6: return pipe_kernel_launch<6>(p, f, zt, part, part_bytes, st);
    case 8: return pipe_kernel_launch<8>(p, f, zt, part, part_bytes, st);
    case 10: return pipe_kernel_launch<10>(p, f, zt, part, part_bytes, st);
    case 12: return pipe_kernel_launch<12>(p, f, zt, part, part_bytes, st);
    case 14: return pipe_kernel_launch<14>(p, f, zt, part, part_bytes, st);
    case 16: return pipe_kernel_launch<16>(p, f, zt, part, part_bytes, st);
    case 18: return pipe_kernel_launch<18>(p, f, zt, part, part_bytes, st);
    case 20: return pipe_kernel_launch<20>(p, f, zt, part, part_bytes, st);
    case 24: return pipe_kernel_launch<24>(p, f, zt, part, part_bytes, st);
    default: return hipErrorNotSupported;
  }
}

template <typename T, int PF, int GPT>
static hipError_t fused_dispatch(const DftPlan& p, FusedShape& f, const void* zt, void* part, size_t part_bytes,
                                 hipStream_t st) {
  switch (f.fmx) {
    case 1: return fused_kernel_launch<T, PF, GPT, 1>(p, f, zt, part, part_bytes, st);
    case 2: return fused_kernel_launch<T, PF, GPT, 2>(p, f, zt, part, part_bytes, st);
    case 3: return fused_kernel_launch<T, PF, GPT, 3>(p, f, zt, part, part_bytes, st);
    default: return fused_kernel_launch<T, PF, GPT, 4>(p, f, zt, part, part_bytes, st);
  }
}

template <typename T>
static hipError_t fused_launch(const DftPlan& p, const void* zt, void* part, size_t part_bytes, void* zg,
                               const double* scale, hipStream_t st) {
  if (sizeof(T) == 4 && p.pipe) {
    PipeShape ps;
    const hipError_t e = pipe_launch(p, ps, zt, part, part_bytes, st);
    if (e == hipSuccess)
      hipLaunchKernelGGL(dft_zsum_kernel<T>, dim3(cdiv(p.ng, 256), p.nmu), dim3(256), 0, st, (const cx<T>*)part,
                         ps.pmax, (long)p.nmu * p.n2, ps.g, p.n2, p.nmu, p.ng, scale, (cx<T>*)zg);
    if (e != hipErrorNotSupported) return e == hipSuccess ? hipGetLastError() : e;
  }
  FusedShape f;
  if (!fused_shape<T>(p, f)) return hipErrorNotSupported;
  const hipError_t e = (f.pf <= FUSED_PF_S && f.gpt <= FUSED_GPT_S)
                           ? fused_dispatch<T, FUSED_PF_S, FUSED_GPT_S>(p, f, zt, part, part_bytes, st)
                           : fused_dispatch<float, FUSED_PF_L, FUSED_GPT_L>(p, f, zt, part, part_bytes, st);  // FP32 only
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dft_zsum_kernel<T>, dim3(cdiv(p.ng, 256), p.nmu), dim3(256), 0, st, (const cx<T>*)part, f.pmax,
                     (long)p.nmu * p.n2, f.g, p.n2, p.nmu, p.ng, scale, (cx<T>*)zg);
  return hipGetLastError();
}

bool dft_fused_fits(Prec compute, const DftPlan& p) {
  FusedShape f;
  return compute == P64 ? fused_shape<double>(p, f) : fused_shape<float>(p, f);
}

hipError_t dft_fused(Prec compute, const DftPlan& p, const void* zt, void* part, size_t part_bytes, void* zg,
                     const double* scale, hipStream_t st) {
  if (compute == P64) return fused_launch<double>(p, zt, part, part_bytes, zg, scale, st);
  return fused_launch<float>(p, zt, part, part_bytes, zg, scale, st);
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
