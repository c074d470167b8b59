// Step 1 and step 2 contractions with operands generated on the fly.
//
// zpair:  out(mu, c) = conj(Pv(mu, c)) * Qc(mu, c), the least-squares right-hand
//   side of the ISDF fit in factored form (Hadamard product of two orbital
//   Gram blocks): Pv = conj(Psi_v(r_mu)) Psi_v^T, Qc = conj(Psi_c(r_mu)) Psi_c^T.
//   Both blocks are accumulated in registers by one kernel (two K phases) and
//   multiplied in the epilogue, so neither Gram block ever reaches HBM.
//
// core:  M(mu, nu) = sum_{i in v, j in c} C(mu; i, j) w_ij conj(C(nu; i, j)) with
//   C(mu; i, j) = conj(psi_i(r_mu)) psi_j(r_mu) (eq. COmegaCstar): a HERK with
//   K = Nv Nc whose operands are built tile by tile in LDS from the orbitals at
//   the points (Khatri-Rao on the fly), never stored.  Only lower tiles are
//   computed (mirrored), and the occupied index is split across workgroups with
//   a deterministic fixed-order reduction.
#include "internal.h"
#include "kmajor.h"
#include "tile.h"

#include <algorithm>
#include <cmath>

namespace isdf {

// ----------------------------------------------------------------------------
// shared K loop: acc += A(m, k) B(k, n) over [0, K) with x-contiguous operands
// ----------------------------------------------------------------------------
template <typename T, typename S, class TL>
__device__ __forceinline__ void kloop_xx(cx<T>* smem, const cx<S>* A, long lda, const cx<S>* B, long ldb,
                                         int m0, int n0, int M, int N, int K, T ca, T cb,
                                         typename TL::acc_t (&acc)[TL::FM][TL::FN], int tid,
                                         int wm0, int wn0, int lane) {
  Stager<T, S, TL::BM, TL::BK, TL::NT, true> sa;
  Stager<T, S, TL::BN, TL::BK, TL::NT, true> sb;
  const int nk = (K + TL::BK - 1) / TL::BK;
  if (nk == 0) return;
  sa.fetch(A, 1, lda, m0, 0, M, K, tid);
  sb.fetch(B, 1, ldb, n0, 0, N, K, tid);
  __syncthreads();
  sa.store(smem, TL::LDA, ca, tid);
  sb.store(smem + TL::AS, TL::LDB, cb, tid);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) {
      sa.fetch(A, 1, lda, m0, (kt + 1) * TL::BK, M, K, tid);
      sb.fetch(B, 1, ldb, n0, (kt + 1) * TL::BK, N, K, tid);
    }
    cx<T>* sc = smem + cur * (TL::AS + TL::BS);
    cx<T>* sn = smem + (cur ^ 1) * (TL::AS + TL::BS);
    tile_mma<T, TL>(sc, sc + TL::AS, acc, wm0, wn0, lane);
    if (kt + 1 < nk) {
      sa.store(sn, TL::LDA, ca, tid);
      sb.store(sn + TL::AS, TL::LDB, cb, tid);
    }
    __syncthreads();
  }
}

template <typename T, typename S, typename SO, class TL>
__global__ __launch_bounds__(TL::NT) void zpair_kernel(int M, int N, int nv, int ns, int b0, const cx<S>* pm,
                                                       long ldp, const cx<S>* b, long ldb, SO* out,
                                                       long ldo, int ntm, int total, int herm) {
  __shared__ cx<T> smem[2 * (TL::AS + TL::BS)];
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  int bm = id % ntm, bn = id / ntm;
  if (herm) {   // Hermitian output (b = pm): lower-triangle tiles bn <= bm, row-major
    int r = (int)((sqrt(8.0 * id + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > id) --r;
    while ((r + 1) * (r + 2) / 2 <= id) ++r;
    bm = r;
    bn = id - r * (r + 1) / 2;
  }
  const int m0 = bm * TL::BM, n0 = bn * TL::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % TL::WGM) * TL::WTM, wn0 = (wave / TL::WGM) * TL::WTN;

  typename TL::acc_t accp[TL::FM][TL::FN], accq[TL::FM][TL::FN];
  zero_acc<TL>(accp);
  zero_acc<TL>(accq);
  kloop_xx<T, S, TL>(smem, pm, ldp, b, ldb, m0, n0, M, N, nv, (T)-1, (T)1, accp, tid, wm0, wn0, lane);
  kloop_xx<T, S, TL>(smem, pm + (long)b0 * ldp, ldp, b + (long)b0 * ldb, ldb, m0, n0, M, N, ns - nv,
                     (T)-1, (T)1, accq, tid, wm0, wn0, lane);

  const int rc = lane & 15, part = rc & 1;
#pragma unroll
  for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T po = accp[fm][fn][v], qo = accq[fm][fn][v];
        const T px = xor1(po), qx = xor1(qo);
        // conj(P) Q: re = Pr Qr + Pi Qi, im = Pr Qi - Pi Qr
        const T val = part == 0 ? (po * qo + px * qx) : (px * qo - po * qx);
        const int row = m0 + wm0 + fm * 16 + Mfma<T>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        if (row < M && col < N) {
          out[((long)row * ldo + col) * 2 + part] = (SO)val;
          if (herm && bm != bn) out[((long)col * ldo + row) * 2 + part] = (SO)(part ? -val : val);   // mirrored
        }
      }
}

// ----------------------------------------------------------------------------
// Single-precision pair kernel: 128 points x 64 grid columns per workgroup on
// the k-major engine of kmajor.h; the occupied K tiles accumulate into P and the
// empty ones into Q in one pipeline.
// ----------------------------------------------------------------------------
// Generic K loop (any tile edge): clamped loads, masked LDS stores.
__device__ __forceinline__ void zl_loop_generic(float* smem, int M, int N, int nv, int ns, int b0, const c32* pm,
                                                long ldp, const z64* b, long ldb, int m0, int n0,
                                                f4 (&accp)[ZL::FM][ZL::FN], f4 (&accq)[ZL::FM][ZL::FN],
                                                int tid, int wm0, int wn0, int lane) {
  const int tp = (nv + ZL::BK - 1) / ZL::BK, tq = (ns - nv + ZL::BK - 1) / ZL::BK;
  const int nt = tp + tq;
  auto kbase = [&](int t, const c32*& pa, const z64*& pb, int& k0, int& K) {
    if (t < tp) { pa = pm; pb = b; k0 = t * ZL::BK; K = nv; }
    else { pa = pm + (long)b0 * ldp; pb = b + (long)b0 * ldb; k0 = (t - tp) * ZL::BK; K = ns - nv; }
  };
  Stager<float, float, ZL::BM, ZL::BK, ZL::NT, true> sa;
  Stager<float, double, ZL::BN, ZL::BK, ZL::NT, true> sb;   // orbitals rounded to FP32 at staging
  {
    const c32* pa; const z64* pb; int k0, K;
    kbase(0, pa, pb, k0, K);
    sa.fetch(pa, 1, ldp, m0, k0, M, K, tid);
    sb.fetch(pb, 1, ldb, n0, k0, N, K, tid);
    sa.store(reinterpret_cast<c32*>(smem), ZL::LDA, -1.f, tid);
    store_b4(sb, smem + ZL::AS, ZL::LDB, 1.f, tid);
  }
  __syncthreads();
  for (int t = 0; t < nt; ++t) {
    const int cur = t & 1;
    if (t + 1 < nt) {
      const c32* pa; const z64* pb; int k0, K;
      kbase(t + 1, pa, pb, k0, K);
      sa.fetch(pa, 1, ldp, m0, k0, M, K, tid);
      sb.fetch(pb, 1, ldb, n0, k0, N, K, tid);
    }
    const float* sc = smem + cur * (ZL::AS + ZL::BS);
    if (t < tp) zl_mma(sc, sc + ZL::AS, accp, wm0, wn0, lane);
    else zl_mma(sc, sc + ZL::AS, accq, wm0, wn0, lane);
    if (t + 1 < nt) {
      float* sn = smem + (cur ^ 1) * (ZL::AS + ZL::BS);
      sa.store(reinterpret_cast<c32*>(sn), ZL::LDA, -1.f, tid);
      store_b4(sb, sn + ZL::AS, ZL::LDB, 1.f, tid);
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void zl_epilogue(float* out, long ldo, int M, int N, int m0, int n0,
                                            const f4 (&accp)[ZL::FM][ZL::FN], const f4 (&accq)[ZL::FM][ZL::FN],
                                            int wm0, int wn0, int lane) {
  const int rc = lane & 15, part = rc & 1;
#pragma unroll
  for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < ZL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const float po = accp[fm][fn][v], qo = accq[fm][fn][v];
        const float px = xor1(po), qx = xor1(qo);
        // conj(P) Q: re = Pr Qr + Pi Qi, im = Pr Qi - Pi Qr
        const float val = part == 0 ? (po * qo + px * qx) : (px * qo - po * qx);
        const int row = m0 + wm0 + fm * 16 + Mfma<float>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        // streaming store: Z is written once and read back only by the next stage, so it
        // should not push the operand panels, which the XCD's other tiles still read, out of L2
        if (row < M && col < N) __builtin_nontemporal_store(val, out + ((long)row * ldo + col) * 2 + part);
      }
}

// Interior-tile fetch of the pair kernel: the points (A) as complex64 like
// ZFetch, the orbitals (B) straight from their complex128 storage, two values
// (32 bytes) per thread, rounded to FP32 as they are staged.  No converted copy
// of the orbitals is made.
struct ZFetchB64 {
  uint32_t aoff0, aoff1, boff;
  int ax, ak, bx, bk;
  int tsplit;    // first K tile of the second state range
  long shift;    // rows from K tile tsplit's position to the second range's first state
  f4 ra0, ra1;
  d4 rb;
  __device__ __forceinline__ void init(int tid, long ldp, long ldb) {
    ax = 2 * (tid & 63); ak = tid >> 6; bx = 2 * (tid & 31); bk = tid >> 5;
    aoff0 = (uint32_t)((ak * ldp + ax) * 8);
    aoff1 = (uint32_t)(((ak + 8) * ldp + ax) * 8);
    boff = (uint32_t)((bk * ldb + bx) * 16);
  }
  __device__ __forceinline__ void fetch(const c32* pm, long ldp, const z64* b, long ldb, int m0, int n0, int t) {
    const long kr = (long)t * ZL::BK + (t >= tsplit ? shift : 0);
    const char* pa = reinterpret_cast<const char*>(pm + kr * ldp + m0);
    const char* pb = reinterpret_cast<const char*>(b + kr * ldb + n0);
    ra0 = *reinterpret_cast<const f4*>(pa + aoff0);
    ra1 = *reinterpret_cast<const f4*>(pa + aoff1);
    rb = *reinterpret_cast<const d4*>(pb + boff);
  }
  __device__ __forceinline__ void stage(float* buf, float sa, float sb) const {
    *reinterpret_cast<f4*>(buf + (ak * ZL::LDA + ax) * 2) = f4{ra0[0], sa * ra0[1], ra0[2], sa * ra0[3]};
    *reinterpret_cast<f4*>(buf + ((ak + 8) * ZL::LDA + ax) * 2) = f4{ra1[0], sa * ra1[1], ra1[2], sa * ra1[3]};
    float* bb = buf + ZL::AS + (bk * ZL::LDB + bx) * 4;
    const float r0 = (float)rb[0], i0 = sb * (float)rb[1], r1 = (float)rb[2], i1 = sb * (float)rb[3];
    *reinterpret_cast<f4*>(bb) = f4{r0, i0, -i0, r0};
    *reinterpret_cast<f4*>(bb + 4) = f4{r1, i1, -i1, r1};
  }
};

// Interior tiles (nti x ntj of them, all full): one workgroup per CU walks its
// share with no inter-workgroup synchronisation.  The tiles of each XCD form a
// contiguous range of the point-fastest tile order, dealt to that XCD's
// workgroups in turn, so they share the grid-orbital panels in its L2.  The
// occupied and the empty K ranges run through one K loop with one running
// accumulator, whose occupied sum moves to accp at the boundary.  EVEN (both
// ranges an even number of K tiles): the first K tile is staged before the tile
// loop and each range's last K tile stages the next range's first one, so no
// range starts with a wait on global loads; the refill loads would otherwise be
// waited for behind the previous tile's Z stores, which the memory counter
// retires in issue order.
template <bool EVEN>
__global__ __launch_bounds__(ZL::NT) __attribute__((amdgpu_waves_per_eu(3)))
void zpair32_kernel(int nv, int ns, int b0, const c32* pm, long ldp, const z64* b, long ldb, float* out, long ldo,
                    int nti, int total) {
  __shared__ float smem[2 * (ZL::AS + ZL::BS)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % ZL::WGM) * ZL::WTM, wn0 = (wave / ZL::WGM) * ZL::WTN;
  const int xcd = blockIdx.x % 8, nper = gridDim.x / 8, j = blockIdx.x / 8;
  const int per = (total + 7) / 8;
  const int lo = xcd * per, hi = min(total, lo + per);
  const int tp = nv / ZL::BK, nt = ns / ZL::BK;
  ZFetchB64 zf;
  ZFrag frag[2];
  zf.init(tid, ldp, ldb);
  zf.tsplit = tp;
  zf.shift = (long)b0 - nv;
  if (lo + j < hi) {
    zf.fetch(pm, ldp, b, ldb, ((lo + j) % nti) * ZL::BM, ((lo + j) / nti) * ZL::BN, 0);
    if (EVEN) {   // every range then starts staged
      zf.stage(smem, -1.f, 1.f);
      __syncthreads();
      zl_frag(smem, 0, frag[0], wm0, wn0, lane);
    }
  }
  for (int id = lo + j; id < hi; id += nper) {
    const int m0 = (id % nti) * ZL::BM, n0 = (id / nti) * ZL::BN;
    const int nid = id + nper;
    f4 accp[ZL::FM][ZL::FN], accq[ZL::FM][ZL::FN];
#pragma unroll
    for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < ZL::FN; ++fn) accq[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
    for (int ph = 0; ph < 2; ++ph) {
      const bool last = ph == 1;
      zl_range(smem, zf, frag, last ? tp : 0, last ? nt : tp, EVEN, -1.f, 1.f, pm,
               ldp, b, ldb, m0, n0, last ? nid < hi : true, last ? (nid % nti) * ZL::BM : m0,
               last ? (nid / nti) * ZL::BN : n0, last ? 0 : tp, accq, wm0, wn0, lane);
      if (!last) {
#pragma unroll
        for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < ZL::FN; ++fn) {
            accp[fm][fn] = accq[fm][fn];
            accq[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
          }
      }
    }
    zl_epilogue(out, ldo, (m0 + ZL::BM), (n0 + ZL::BN), m0, n0, accp, accq, wm0, wn0, lane);
  }
}

// Any tiles (edges, or operands that do not allow the 16-byte path): one
// workgroup per tile from a list given as (first tile, count) of a column-major
// walk over the ntm x ntn tiles, or the edge strips.
__global__ __launch_bounds__(ZL::NT) void zpair32_edge_kernel(int M, int N, int nv, int ns, int b0, const c32* pm,
                                                              long ldp, const z64* b, long ldb, float* out,
                                                              long ldo, int ntm, int ntn, int nti, int ntj,
                                                              int all) {
  __shared__ float smem[2 * (ZL::AS + ZL::BS)];
  int bm, bn;
  const int e = blockIdx.x;
  if (all) {
    bm = e % ntm; bn = e / ntm;
  } else if (ntj < ntn && e < ntm) {  // last (partial) column strip, every row
    bm = e; bn = ntj;
  } else {                            // last (partial) row strip, interior columns
    const int r = (ntj < ntn) ? e - ntm : e;
    bm = nti; bn = r;
  }
  if (bm >= ntm || bn >= ntn) return;
  const int m0 = bm * ZL::BM, n0 = bn * ZL::BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % ZL::WGM) * ZL::WTM, wn0 = (wave / ZL::WGM) * ZL::WTN;
  f4 accp[ZL::FM][ZL::FN], accq[ZL::FM][ZL::FN];
#pragma unroll
  for (int fm = 0; fm < ZL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < ZL::FN; ++fn) accp[fm][fn] = accq[fm][fn] = f4{0.f, 0.f, 0.f, 0.f};
  zl_loop_generic(smem, M, N, nv, ns, b0, pm, ldp, b, ldb, m0, n0, accp, accq, tid, wm0, wn0, lane);
  zl_epilogue(out, ldo, M, N, m0, n0, accp, accq, wm0, wn0, lane);
}

static hipError_t zpair32_launch(int M, int N, int nv, int ns, int b0, const void* pm, long ldp, const void* b,
                                 long ldb, void* out, long ldo, hipStream_t st, int wg_per_cu) {
  const int ntm = (int)cdiv(M, ZL::BM), ntn = (int)cdiv(N, ZL::BN);
  if (ntm == 0 || ntn == 0) return hipSuccess;
  // the vector-load interior path needs K tiles that never straddle the occupied /
  // empty boundary, even leading dimensions, a 16-byte aligned point base and a
  // 32-byte aligned orbital base
  const bool aligned = nv % ZL::BK == 0 && (ns - nv) % ZL::BK == 0 && (ldp & 1) == 0 && (ldb & 1) == 0 &&
                       (reinterpret_cast<uintptr_t>(pm) & 15) == 0 && (reinterpret_cast<uintptr_t>(b) & 31) == 0;
  const int nti = aligned ? M / ZL::BM : 0, ntj = aligned ? N / ZL::BN : 0;
  const int interior = nti * ntj;
  if (interior > 0) {
    // wg_per_cu workgroups per CU (a multiple of 8: one share per XCD), never more than the tiles
    const int wpc = std::max(1, std::min(wg_per_cu, 4));
    const int g = std::max(8, std::min(8 * ((wpc * cu_count() + 7) / 8), 8 * (int)cdiv(interior, 8)));
    const int tp = nv / ZL::BK, tq = (ns - nv) / ZL::BK;
    if (tp >= 2 && tp % 2 == 0 && tq >= 2 && tq % 2 == 0)
      hipLaunchKernelGGL(zpair32_kernel<true>, dim3(g), dim3(ZL::NT), 0, st, nv, ns, b0, (const c32*)pm, ldp,
                         (const z64*)b, ldb, (float*)out, ldo, nti, interior);
    else
      hipLaunchKernelGGL(zpair32_kernel<false>, dim3(g), dim3(ZL::NT), 0, st, nv, ns, b0, (const c32*)pm, ldp,
                         (const z64*)b, ldb, (float*)out, ldo, nti, interior);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int all = interior == 0 ? 1 : 0;
  const int nedge = all ? ntm * ntn : (ntj < ntn ? ntm : 0) + (nti < ntm ? ntj : 0);
  if (nedge == 0) return hipSuccess;
  hipLaunchKernelGGL(zpair32_edge_kernel, dim3(nedge), dim3(ZL::NT), 0, st, M, N, nv, ns, b0, (const c32*)pm,
                     ldp, (const z64*)b, ldb, (float*)out, ldo, ntm, ntn, nti, ntj, all);
  return hipGetLastError();
}

typedef Tile<double, 64, 64, 16, 2, 2> TZ64;
// Small FP64 products (fewer 64 x 64 tiles than CUs, e.g. S at the points): 32 x 32
// tiles, four times the workgroups, each light enough to share a CU with a
// compute-bound kernel on another stream.  The k order per output element is that
// of the 64 x 64 tile, so the results are the same.
typedef Tile<double, 32, 32, 16, 2, 2> TZ64S;

// FP64 pair kernel on the grid, persistent: one workgroup per slot walks its XCD's
// contiguous share of the 64 x 64 tiles in point-fastest order (consecutive tiles
// share the grid-orbital panel in that XCD's L2).  The occupied and the empty K
// ranges run through one K loop with one running accumulator, whose occupied sum
// moves to accp at the range boundary; the loop fetches the next K tile (or the
// next tile's first one) into registers while the MFMAs of the current one run,
// so no tile starts with an exposed load.  Needs no tile edges: M % 64 == 0,
// N % 64 == 0 (the caller keeps zpair_kernel for anything else).
typedef Tile<double, 64, 64, 16, 4, 2> TZ64P;   // 8 waves of 16 x 32 (the generic 4-wave tile needs 315 registers)

__global__ __launch_bounds__(TZ64P::NT, 1) void zpair64_kernel(int nv, int ns, int b0, const z64* __restrict__ pm,
                                                               long ldp, const z64* __restrict__ b, long ldb,
                                                               z64* __restrict__ out, long ldo, int nti, int total) {
  typedef TZ64P TL;
  __shared__ z64 smem[2 * (TL::AS + TL::BS)];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % TL::WGM) * TL::WTM, wn0 = (wave / TL::WGM) * TL::WTN;
  const int xcd = blockIdx.x % 8, nper = gridDim.x / 8, j = blockIdx.x / 8;
  const int per = (total + 7) / 8;
  const int lo = xcd * per, hi = min(total, lo + per);
  const int tp = (nv + TL::BK - 1) / TL::BK, tq = (ns - nv + TL::BK - 1) / TL::BK, nt = tp + tq;
  const int K1 = ns - nv;
  Stager<double, double, TL::BM, TL::BK, TL::NT, true> sa;
  Stager<double, double, TL::BN, TL::BK, TL::NT, true> sb;
  // K tile t of the tile at (m0, n0): the occupied range, then the second range from row b0
  auto fetch = [&](int t, int m0, int n0) {
    if (t < tp) {
      sa.fetch(pm, 1, ldp, m0, t * TL::BK, 1 << 30, nv, tid);
      sb.fetch(b, 1, ldb, n0, t * TL::BK, 1 << 30, nv, tid);
    } else {
      sa.fetch(pm + (long)b0 * ldp, 1, ldp, m0, (t - tp) * TL::BK, 1 << 30, K1, tid);
      sb.fetch(b + (long)b0 * ldb, 1, ldb, n0, (t - tp) * TL::BK, 1 << 30, K1, tid);
    }
  };
  auto stage = [&](int s) {
    z64* buf = smem + s * (TL::AS + TL::BS);
    sa.store(buf, TL::LDA, -1.0, tid);
    sb.store(buf + TL::AS, TL::LDB, 1.0, tid);
  };
  int id = lo + j;
  if (id < hi) {
    fetch(0, (id % nti) * TL::BM, (id / nti) * TL::BN);
    stage(0);
  }
  __syncthreads();
  int cur = 0;
  const int rc = lane & 15, part = rc & 1;
  for (; id < hi; id += nper) {
    const int m0 = (id % nti) * TL::BM, n0 = (id / nti) * TL::BN;
    const int nid = id + nper;
    TL::acc_t acc[TL::FM][TL::FN], accp[TL::FM][TL::FN];
    zero_acc<TL>(acc);
    for (int t = 0; t < nt; ++t) {
      const bool last = t + 1 == nt;
      if (!last) fetch(t + 1, m0, n0);
      else if (nid < hi) fetch(0, (nid % nti) * TL::BM, (nid / nti) * TL::BN);
      const z64* buf = smem + cur * (TL::AS + TL::BS);
      tile_mma<double, TL>(buf, buf + TL::AS, acc, wm0, wn0, lane);
      if (t + 1 == tp) {
#pragma unroll
        for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
          for (int fn = 0; fn < TL::FN; ++fn) {
            accp[fm][fn] = acc[fm][fn];
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[fm][fn][v] = 0.0;
          }
      }
      if (!last || nid < hi) stage(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
    double* o = reinterpret_cast<double*>(out);
#pragma unroll
    for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double po = accp[fm][fn][v], qo = acc[fm][fn][v];
          const double px = xor1(po), qx = xor1(qo);
          // conj(P) Q: re = Pr Qr + Pi Qi, im = Pr Qi - Pi Qr
          const double val = part == 0 ? (po * qo + px * qx) : (px * qo - po * qx);
          const int row = m0 + wm0 + fm * 16 + Mfma<double>::row(lane, v);
          const int col = n0 + wn0 + fn * 8 + (rc >> 1);
          o[((long)row * ldo + col) * 2 + part] = val;
        }
  }
}

template <typename T, typename S, typename SO, class TL>
static hipError_t zpair_launch(int M, int N, int nv, int ns, int b0, const void* pm, long ldp, const void* b,
                               long ldb, void* out, long ldo, hipStream_t st, bool herm = false) {
  const int ntm = (int)cdiv(M, TL::BM), ntn = (int)cdiv(N, TL::BN);
  const int total = herm ? ntm * (ntm + 1) / 2 : ntm * ntn;
  if (total == 0) return hipSuccess;
  const unsigned grid = 8u * (unsigned)((total + 7) / 8);
  hipLaunchKernelGGL((zpair_kernel<T, S, SO, TL>), dim3(grid), dim3(TL::NT), 0, st, M, N, nv, ns, b0,
                     (const cx<S>*)pm, ldp, (const cx<S>*)b, ldb, (SO*)out, ldo, ntm, total, herm ? 1 : 0);
  return hipGetLastError();
}

hipError_t zpair(Prec compute, int M, int N, int nv, int ns, const void* pm, long ldp, const void* b,
                 long ldb, bool in32, void* out, long ldo, bool out32, hipStream_t st, int wg_per_cu, int b0) {
  if (b0 < 0) b0 = nv;   // the second state range follows the first
  if (compute == P64) {
    if (out32 || in32) return hipErrorInvalidValue;
    const int nti = M / TZ64P::BM, ntj = N / TZ64P::BN;
    const long total = (long)nti * ntj;
    if (M % TZ64P::BM == 0 && N % TZ64P::BN == 0 && nv >= 1 && ns > nv && total >= 8 * cu_count()) {
      // persistent: one 8-wave workgroup per CU (207 registers: two waves per SIMD), a
      // multiple of 8 (one share per XCD)
      const int g = (int)std::min<long>(8L * ((cu_count() + 7) / 8), 8L * ((total + 7) / 8));
      hipLaunchKernelGGL(zpair64_kernel, dim3(g), dim3(TZ64P::NT), 0, st, nv, ns, b0, (const z64*)pm, ldp,
                         (const z64*)b, ldb, (z64*)out, ldo, nti, (int)total);
      return hipGetLastError();
    }
    // the same operands on both sides (S at the points): Hermitian, lower tiles only
    const bool herm = pm == b && M == N && ldp == ldb;
    if (cdiv(M, TZ64::BM) * cdiv(N, TZ64::BN) < cu_count())
      return zpair_launch<double, double, double, TZ64S>(M, N, nv, ns, b0, pm, ldp, b, ldb, out, ldo, st, herm);
    return zpair_launch<double, double, double, TZ64>(M, N, nv, ns, b0, pm, ldp, b, ldb, out, ldo, st, herm);
  }
  // single precision: complex64 points, complex128 orbitals (rounded as staged), complex64 output
  if (!in32 || !out32) return hipErrorInvalidValue;
  return zpair32_launch(M, N, nv, ns, b0, pm, ldp, b, ldb, out, ldo, st, wg_per_cu);
}

// ----------------------------------------------------------------------------
// core
// ----------------------------------------------------------------------------
template <typename T, class TL>
__global__ __launch_bounds__(TL::NT) void core_kernel(int nmu, int nv, int nc, const z64* pm, long ldp,
                                                      const double* w, cx<T>* part, int nsplit,
                                                      int total) {
  __shared__ cx<T> smem[2 * (TL::AS + TL::BS)];
  static_assert(TL::BM == TL::BN, "square tiles");
  static_assert(TL::NT % TL::BM == 0, "thread map");
  const int id = xcd_remap(blockIdx.x, total);
  if (id >= total) return;
  int r = (int)((sqrt(8.0 * id + 1.0) - 1.0) * 0.5);
  while (r * (r + 1) / 2 > id) --r;
  while ((r + 1) * (r + 2) / 2 <= id) ++r;
  const int bm = r, bn = id - r * (r + 1) / 2;
  const int m0 = bm * TL::BM, n0 = bn * TL::BN;
  const int split = blockIdx.y;
  w += (long)blockIdx.z * nv * nc;                        // weight set of this batch item
  part += (long)blockIdx.z * nsplit * nmu * nmu;
  const int i0 = (int)((long)split * nv / nsplit), i1 = (int)((long)(split + 1) * nv / nsplit);
  const int ni = i1 - i0;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm0 = (wave % TL::WGM) * TL::WTM, wn0 = (wave / TL::WGM) * TL::WTN;

  // thread map: x = tid % BM (point within tile), kk = tid / BM + e * (NT / BM)
  constexpr int KSTEP = TL::NT / TL::BM;
  constexpr int E = TL::BK / KSTEP;
  const int x = tid % TL::BM, kb = tid / TL::BM;
  const int gm = m0 + x, gn = n0 + x;
  const bool okm = gm < nmu, okn = gn < nmu;
  const z64* pc = pm + (long)nv * ldp;

  const int njc = (nc + TL::BK - 1) / TL::BK;
  const int S = njc * ni;
  // Raw operands of the next stage, loaded before the MFMA step of the current
  // one (addresses clamped to valid memory, masked when formed).
  z64 bm_raw[E], bn_raw[E];   // b_j at this thread's points (reloaded when the j block changes)
  double w_raw[E];
  z64 am_raw, an_raw;
  int cur_jc = -1, nxt_jc = 0;
  const long pmo = okm ? gm : 0, pno = okn ? gn : 0;

  auto fetch = [&](int s) {
    const int jc = s / ni, i = i0 + s % ni;
    if (jc != cur_jc) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int j = jc * TL::BK + kb + e * KSTEP;
        const long jo = (j < nc) ? (long)j * ldp : 0;
        bm_raw[e] = pc[jo + pmo];
        bn_raw[e] = pc[jo + pno];
      }
      cur_jc = jc;
    }
    nxt_jc = jc;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = jc * TL::BK + kb + e * KSTEP;
      w_raw[e] = w[(long)i * nc + ((j < nc) ? j : 0)];
    }
    am_raw = pm[(long)i * ldp + pmo];
    an_raw = pm[(long)i * ldp + pno];
  };
  auto store = [&](cx<T>* buf) {
    const cx<T> am = okm ? cvt<T>(am_raw) : cx<T>{0, 0};
    const cx<T> an = okn ? cvt<T>(an_raw) : cx<T>{0, 0};
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int kk = kb + e * KSTEP;
      const bool okj = nxt_jc * TL::BK + kk < nc;
      const T wij = okj ? (T)w_raw[e] : (T)0;
      const cx<T> bmv = okm ? cvt<T>(bm_raw[e]) : cx<T>{0, 0};
      const cx<T> bnv = okn ? cvt<T>(bn_raw[e]) : cx<T>{0, 0};
      const cx<T> t = cmulc(am, bmv);                       // conj(a_i(mu)) b_j(mu)
      buf[kk * TL::LDA + x] = cx<T>{t.re * wij, t.im * wij};
      const cx<T> u = cmul(an, cconj(bnv));                 // a_i(nu) conj(b_j(nu))
      buf[TL::AS + kk * TL::LDB + x] = okj ? u : cx<T>{0, 0};
    }
  };

  // Single precision: the MFMA accumulators hold at most FLUSH k tiles
  // (FLUSH * BK terms) before they are added into FP64 registers, so the FP32
  // accumulation error stays that of a short sum however long K = Nv Nc is.
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int FLUSH = 16;
  typename TL::acc_t acc[TL::FM][TL::FN];
  double acc64[TL::FM][TL::FN][4];
  zero_acc<TL>(acc);
#pragma unroll
  for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[fm][fn][v] = 0.0;
  auto flush = [&]() {
#pragma unroll
    for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
      for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc64[fm][fn][v] += (double)acc[fm][fn][v];
          acc[fm][fn][v] = (T)0;
        }
  };
  if (S > 0) {
    fetch(0);
    store(smem);
    __syncthreads();
    for (int s = 0; s < S; ++s) {
      const int cur = s & 1;
      if (s + 1 < S) fetch(s + 1);
      cx<T>* sc = smem + cur * (TL::AS + TL::BS);
      tile_mma<T, TL>(sc, sc + TL::AS, acc, wm0, wn0, lane);
      if (F32 && (s + 1) % FLUSH == 0) flush();
      if (s + 1 < S) store(smem + (cur ^ 1) * (TL::AS + TL::BS));
      __syncthreads();
    }
  }
  if (F32) flush();

  T* out = reinterpret_cast<T*>(part + (long)split * nmu * nmu);
  const int rc = lane & 15, pp = rc & 1;
#pragma unroll
  for (int fm = 0; fm < TL::FM; ++fm)
#pragma unroll
    for (int fn = 0; fn < TL::FN; ++fn)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = m0 + wm0 + fm * 16 + Mfma<T>::row(lane, v);
        const int col = n0 + wn0 + fn * 8 + (rc >> 1);
        if (row >= nmu || col >= nmu) continue;
        const double a = F32 ? acc64[fm][fn][v] : (double)acc[fm][fn][v];
        const T val = (row == col && pp == 1) ? (T)0 : (T)a;  // Hermitian: real diagonal
        if (bm == bn && row < col) continue;
        out[((long)row * nmu + col) * 2 + pp] = val;
        if (row > col) out[((long)col * nmu + row) * 2 + pp] = pp ? -val : val;
      }
}

typedef Tile<double, 64, 64, 16, 2, 2> TC64;
typedef Tile<float, 64, 64, 32, 2, 2> TC32;

int core_splits(int nmu, int nv) {
  const int nt = (nmu + 63) / 64;
  const int tiles = nt * (nt + 1) / 2;
  int s = (1024 + tiles - 1) / tiles;
  if (s > nv) s = nv;
  if (s < 1) s = 1;
  return s;
}

hipError_t core_partial(Prec compute, int nmu, int nv, int nc, const void* pm, long ldp,
                        const double* w, void* part, int nsplit, hipStream_t st, int batch) {
  const int nt = (nmu + 63) / 64;
  const int total = nt * (nt + 1) / 2;
  const unsigned gx = 8u * (unsigned)((total + 7) / 8);
  if (compute == P64) {
    hipLaunchKernelGGL((core_kernel<double, TC64>), dim3(gx, nsplit, batch), dim3(TC64::NT), 0, st, nmu, nv,
                       nc, (const z64*)pm, ldp, w, (z64*)part, nsplit, total);
  } else {
    hipLaunchKernelGGL((core_kernel<float, TC32>), dim3(gx, nsplit, batch), dim3(TC32::NT), 0, st, nmu, nv,
                       nc, (const z64*)pm, ldp, w, (c32*)part, nsplit, total);
  }
  return hipGetLastError();
}

template <typename T>
__global__ void core_reduce_kernel(long n2, const T* part, int nsplit, double scale, double* m_out,
                                   double* negm) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;  // real index over 2 n2
  if (idx >= 2 * n2) return;
  const long b = blockIdx.y;                                       // batch item
  part += b * nsplit * 2 * n2;
  if (m_out) m_out += b * 2 * n2;
  if (negm) negm += b * 2 * n2;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += (double)part[(long)k * 2 * n2 + idx];
  s *= scale;
  if (m_out) m_out[idx] = s;
  if (negm) negm[idx] = -s;
}

hipError_t core_reduce(Prec compute, int nmu, const void* part, int nsplit, double scale, void* m_out,
                       void* negm_out, hipStream_t st, int batch) {
  const long n2 = (long)nmu * nmu;
  const dim3 grid(cdiv(2 * n2, 256), batch);
  if (compute == P64)
    hipLaunchKernelGGL((core_reduce_kernel<double>), dim3(grid), dim3(256), 0, st, n2,
                       (const double*)part, nsplit, scale, (double*)m_out, (double*)negm_out);
  else
    hipLaunchKernelGGL((core_reduce_kernel<float>), grid, dim3(256), 0, st, n2,
                       (const float*)part, nsplit, scale, (double*)m_out, (double*)negm_out);
  return hipGetLastError();
}

}  // namespace isdf
