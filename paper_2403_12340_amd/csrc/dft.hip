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

// LDS rows are padded to an odd number of complex elements so that lanes
// reading different rows hit different banks.
__host__ __device__ inline int odd_pad(int n) { return n | 1; }
__host__ __device__ inline int up16(int n) { return (n + 15) / 16 * 16; }

// x stage as an MFMA product per slab: T1 (y x a) = Z^T-slab (y x x) . TW^T (x x a),
// y up to 64 rows (4 waves of 16), a in chunks of 32 columns, x in 16-deep steps.
template <typename T>
using TileX = Tile<T, 64, 32, 16, 4, 1>;

template <typename T>
static size_t xy_lds_bytes(const DftPlan& p) {
  typedef TileX<T> TL;
  const size_t k16 = up16(p.n0), s1 = odd_pad(p.n1 + 1), sk = odd_pad(p.kx);
  return sizeof(cx<T>) * (k16 * TL::LDA + k16 * TL::LDB + (size_t)p.n1 * sk + (size_t)p.ky * s1);
}

// one workgroup per (z-plane, point)
template <typename T>
__global__ __launch_bounds__(256) void dft_xy_kernel(DftPlan p, const cx<T>* zt, cx<T>* t2) {
  typedef TileX<T> TL;
  extern __shared__ unsigned char lds_raw[];
  const int k16 = up16(p.n0), s1 = odd_pad(p.n1 + 1), sk = odd_pad(p.kx);
  cx<T>* As = reinterpret_cast<cx<T>*>(lds_raw);   // [x][y] slab, k-major A operand
  cx<T>* Bs = As + k16 * TL::LDA;                   // [x][a] twiddle chunk, k-major B operand
  cx<T>* T1 = Bs + k16 * TL::LDB;                   // [y][sk]  after the x stage
  cx<T>* TY = T1 + p.n1 * sk;                       // [ky][s1] y twiddles
  const int z = blockIdx.x, mu = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const long slab = ((long)mu * p.n2 + z) * p.n1 * p.n0;
  const cx<T>* twx = reinterpret_cast<const cx<T>*>(p.twx);
  const cx<T>* twy = reinterpret_cast<const cx<T>*>(p.twy);
  const cx<T> zero{(T)0, (T)0};
  for (int i = tid; i < k16 * 64; i += 256) {       // transpose the slab into [x][y], zero padded
    const int x = i / 64, y = i % 64;
    As[x * TL::LDA + y] = zero;
  }
  __syncthreads();
  for (int i = tid; i < p.n0 * p.n1; i += 256) As[(i % p.n0) * TL::LDA + i / p.n0] = zt[slab + i];
  for (int i = tid; i < p.ky * p.n1; i += 256) TY[(i / p.n1) * s1 + i % p.n1] = twy[i];
  const int wm0 = wave * TL::WTM;
  const int rc = lane & 15, part = rc & 1;
  for (int a0 = 0; a0 < p.kx; a0 += 32) {
    __syncthreads();
    for (int i = tid; i < k16 * 32; i += 256) {
      const int x = i / 32, a = i % 32;
      const bool ok = x < p.n0 && a0 + a < p.kx;
      const cx<T> t = twx[ok ? (a0 + a) * p.n0 + x : 0];
      Bs[x * TL::LDB + a] = cx<T>{ok ? t.re : (T)0, ok ? t.im : (T)0};
    }
    __syncthreads();
    typename TL::acc_t acc[TL::FM][TL::FN];
    zero_acc<TL>(acc);
    for (int kc = 0; kc < k16; kc += 16)
      tile_mma<T, TL>(As + kc * TL::LDA, Bs + kc * TL::LDB, acc, wm0, 0, lane);
    T* T1r = reinterpret_cast<T*>(T1);
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int y = wm0 + Mfma<T>::row(lane, v);
        const int a = a0 + fn * 8 + (rc >> 1);
        if (y < p.n1 && a < p.kx) T1r[(y * sk + a) * 2 + part] = acc[0][fn][v];
      }
  }
  __syncthreads();
  // y stage: only the (x, y) frequency pairs in use
  cx<T>* out = t2 + ((long)mu * p.n2 + z) * p.nd;
  for (int d = tid; d < p.nd; d += 256) {
    const int a = p.d_ax[d], b = p.d_by[d];
    const cx<T>* tw = TY + b * s1;
    T sr = 0, si = 0;
    for (int y = 0; y < p.n1; ++y) {
      const cx<T> v = T1[y * sk + a];
      sr += v.re * tw[y].re - v.im * tw[y].im;
      si += v.re * tw[y].im + v.im * tw[y].re;
    }
    out[d] = cx<T>{sr, si};
  }
}

bool dft_supported(int n0, int n1, int kx, int ky, Prec compute) {
  if (n1 > 64 || n0 > 64) return false;  // one 64-row MFMA tile per slab
  DftPlan p{};
  p.n0 = n0; p.n1 = n1; p.kx = kx; p.ky = ky;
  const size_t bytes = compute == P64 ? xy_lds_bytes<double>(p) : xy_lds_bytes<float>(p);
  return bytes <= 160 * 1024;
}

hipError_t dft_xy(Prec compute, const DftPlan& p, const void* zt, void* t2, hipStream_t st) {
  const dim3 grid(p.n2, p.nmu);
  if (compute == P64) {
    const size_t lds = xy_lds_bytes<double>(p);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dft_xy_kernel<double>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((dft_xy_kernel<double>), grid, dim3(256), lds, st, p, (const z64*)zt, (z64*)t2);
  } else {
    const size_t lds = xy_lds_bytes<float>(p);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&dft_xy_kernel<float>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL((dft_xy_kernel<float>), grid, dim3(256), lds, st, p, (const c32*)zt, (c32*)t2);
  }
  return hipGetLastError();
}

template <typename T>
__global__ void dft_z_kernel(DftPlan p, const cx<T>* t2, cx<T>* zg, const double* scale) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  if (g >= p.ng) return;
  const int d = p.g_d[g], c = p.g_cz[g];
  const cx<T>* twz = reinterpret_cast<const cx<T>*>(p.twz) + (long)c * p.n2;
  const cx<T>* col = t2 + (long)mu * p.n2 * p.nd + d;
  T sr = 0, si = 0;
  for (int z = 0; z < p.n2; ++z) {
    const cx<T> v = col[(long)z * p.nd];
    sr += v.re * twz[z].re - v.im * twz[z].im;
    si += v.re * twz[z].im + v.im * twz[z].re;
  }
  const T sc = scale ? (T)scale[g] : (T)1;
  zg[(long)mu * p.ng + g] = cx<T>{sr * sc, si * sc};
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
