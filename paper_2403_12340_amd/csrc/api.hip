// C ABI of the ISDF-SMW dielectric-inverse library (see include/isdf_smw.h).
//
// Host side only: argument validation, the workspace layout, the pruned-DFT
// index bookkeeping and the order of kernel launches.  Every arithmetic step
// of the method runs in the HIP kernels of this library.
//
// Pipeline of isdf_eps_inv (paper: eq. ISDF, eq. COmegaCstar, eq. epsilon_with_SMW):
//   pm   = psi at the points                                  (gather)
//   S^T  = conj(Pv) * Qc at the points, FP64                  (zpair; S = C C^H)
//   Zt   = (M_vc C^H)^T, N_mu x Nr                            (zpair, mode precision)
//   X^T  = (V^{1/2} F Z)^T on the plane-wave list              (dft_xy, dft_z)
//   G    = X^H X                                              (Hermitian GEMM, split-K)
//   per frequency (side stream, overlapping the above):
//     M  = f C W C^H                                          (core)
//     K  = S M^{-1} S, FP64 sweep of -M and two GEMMs
//   T  = (G - K)^{-1}, FP64 sweep
//   eps~^{-1} = I - (X T) X^H                                 (Hermitian output GEMM)
// Since Theta = Z S^{-1} and U = V^{1/2} F Theta = X S^{-1}, eq. epsilon_with_SMW gives
//   U (M^{-1} - U^H U)^{-1} U^H = X (S M^{-1} S - X^H X)^{-1} X^H,
// so the least-squares fit enters only through S M^{-1} S and S^{-1} is never formed.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <complex>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <deque>
#include <vector>

#include "../../include/isdf_smw.h"
#include "internal.h"

using namespace isdf;

struct isdf_plan_s;

struct isdf_handle_s {
  int device = 0;
  hipStream_t stream = nullptr;   // caller's stream (main branch)
  hipStream_t side = nullptr;     // library-owned stream for the independent branch, default priority
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t ev[10] = {};         // stage timing (main stream)
  hipEvent_t fork = nullptr, join = nullptr, core0 = nullptr, zdone = nullptr, zops = nullptr, tabs = nullptr;
  hipEvent_t mfork = nullptr, mdone = nullptr;  // multi-system calls
  hipEvent_t m_ready[2] = {}, m_used[2] = {};
  std::string err;
};

namespace {

const size_t ALIGN = 256;
inline size_t up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

struct StatusBlock {
  int status;
  int pad;
  double min_pivot;
  double res[10];
  double h2, t2;  // ||H||_F^2 and ||H^{-1}||_F^2 of the last frequency (condition estimate)
  double partial[1024];
};

constexpr int CAUCHY_MAX_NODES = 256;  // contour node table size
constexpr int PLAN_TIMED_CALLS = 256;  // calls a plan times between two syncs
constexpr int CAUCHY_CHUNK = 8;        // nodes per batched Gram pair

struct Problem {
  int n0, n1, n2, nv, nc, ns, nmu, ng, nomega;
  int ngg;         // plane waves the Coulomb Gram runs over: ng, or every grid vector (coulomb_sum = 1)
  bool full_gram;
  int core_method;  // 0: direct pair sum; 1: contour integral (Algorithm 2)
  double core_tol;  // quadrature tolerance of the contour integral
  long nr;
  bool cplx;
  Prec prec;
  bool m32;  // large contractions stored in complex64
  double f, v_scale;
  int refine;
  double recip[9];
  int zrows = 0;   // rows of the Z^T region and the DFT scratch (0: N_mu; the adjoint works in chunks of points)
};

// Points per chunk of the adjoint: the N_mu x Nr intermediates (the pair Gram blocks
// P_a, P_b and Z, and the cotangent of Z) are formed for one chunk of points at a
// time, each at most 512 MiB, in chunks of equal size.
int grad_chunk(const Problem& P) {
  const double per = (double)P.nr * 16.0;                  // bytes of one point's row
  const long cap = std::max<long>(1, (long)((double)(1L << 29) / per));
  const long chunks = (P.nmu + cap - 1) / cap;
  return (int)((P.nmu + chunks - 1) / chunks);
}

// pruned-DFT index lists derived from the Miller list (host bookkeeping)
struct DftIndex {
  std::vector<int> xl, yl, zl, d_ax, d_by, g_d, g_cz, dmap;
  std::vector<int> gd_off, gd_list;   // plane waves grouped by (x, y) pair (CSR, ascending g)
};

DftIndex dft_index(const int32_t* miller, int ng) {
  DftIndex ix;
  auto uniq = [](std::vector<int> v) { std::sort(v.begin(), v.end()); v.erase(std::unique(v.begin(), v.end()), v.end()); return v; };
  std::vector<int> xs(ng), ys(ng), zs(ng);
  std::vector<long> ds(ng);
  auto pairkey = [](int x, int y) { return (long)(x + 1024) * 4096 + (y + 1024); };
  for (int g = 0; g < ng; ++g) {
    xs[g] = miller[3 * g];
    ys[g] = miller[3 * g + 1];
    zs[g] = miller[3 * g + 2];
    ds[g] = pairkey(xs[g], ys[g]);
  }
  ix.xl = uniq(xs);
  ix.yl = uniq(ys);
  ix.zl = uniq(zs);
  std::sort(ds.begin(), ds.end());
  ds.erase(std::unique(ds.begin(), ds.end()), ds.end());
  auto pos = [](const std::vector<int>& v, int x) { return (int)(std::lower_bound(v.begin(), v.end(), x) - v.begin()); };
  for (long k : ds) {
    ix.d_ax.push_back(pos(ix.xl, (int)(k / 4096) - 1024));
    ix.d_by.push_back(pos(ix.yl, (int)(k % 4096) - 1024));
  }
  ix.dmap.assign(ix.xl.size() * ix.yl.size(), -1);
  for (size_t d = 0; d < ix.d_ax.size(); ++d) ix.dmap[(size_t)ix.d_ax[d] * ix.yl.size() + ix.d_by[d]] = (int)d;
  ix.g_d.resize(ng);
  ix.g_cz.resize(ng);
  for (int g = 0; g < ng; ++g) {
    ix.g_d[g] = (int)(std::lower_bound(ds.begin(), ds.end(), pairkey(xs[g], ys[g])) - ds.begin());
    ix.g_cz[g] = pos(ix.zl, zs[g]);
  }
  const size_t nd = ix.d_ax.size();
  ix.gd_off.assign(nd + 1, 0);
  for (int g = 0; g < ng; ++g) ++ix.gd_off[ix.g_d[g] + 1];
  for (size_t d = 0; d < nd; ++d) ix.gd_off[d + 1] += ix.gd_off[d];
  ix.gd_list.resize(ng);
  std::vector<int> fill(ix.gd_off.begin(), ix.gd_off.end() - 1);
  for (int g = 0; g < ng; ++g) ix.gd_list[fill[ix.g_d[g]]++] = g;
  return ix;
}

// Jacobi elliptic functions sn, cn, dn of a real argument u and parameter m in
// [0, 1), and the complete integral K(m), by the arithmetic-geometric mean
// (descending Landen) method of Abramowitz and Stegun 16.4 / 17.6.
struct Jacobi {
  double sn, cn, dn;
};
double ellip_k(double m) {
  double a = 1.0, b = std::sqrt(1.0 - m);
  for (int i = 0; i < 64 && std::fabs(a - b) > 1e-16 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (2.0 * a);
}
Jacobi jacobi_real(double u, double m) {
  if (m <= 0.0) return {std::sin(u), std::cos(u), 1.0};
  double a[40], c[40];
  a[0] = 1.0;
  c[0] = std::sqrt(m);
  double b = std::sqrt(1.0 - m);
  int n = 0;
  while (n < 38 && std::fabs(c[n]) > 1e-17) {
    a[n + 1] = 0.5 * (a[n] + b);
    c[n + 1] = 0.5 * (a[n] - b);
    b = std::sqrt(a[n] * b);
    ++n;
  }
  double phi = std::ldexp(a[n] * u, n), prev = phi;
  for (int k = n; k > 0; --k) {
    prev = phi;
    phi = 0.5 * (phi + std::asin(c[k] * std::sin(phi) / a[k]));
  }
  const double sn = std::sin(phi), cn = std::cos(phi);
  return {sn, cn, n > 0 ? cn / std::cos(prev - phi) : 1.0};
}
// sn, cn, dn at x + i y (real x, y): addition theorem with the imaginary
// transformation (Abramowitz and Stegun 16.21)
void jacobi_complex(double x, double y, double m, std::complex<double>& sn, std::complex<double>& cn,
                    std::complex<double>& dn) {
  const Jacobi r = jacobi_real(x, m), i = jacobi_real(y, 1.0 - m);
  const double den = i.cn * i.cn + m * r.sn * r.sn * i.sn * i.sn;
  sn = std::complex<double>(r.sn * i.dn, r.cn * r.dn * i.sn * i.cn) / den;
  cn = std::complex<double>(r.cn * i.cn, -r.sn * r.dn * i.sn * i.dn) / den;
  dn = std::complex<double>(r.dn * i.cn * i.dn, -m * r.sn * r.cn * i.sn) / den;
}

// Contour of the core's Cauchy integral (Algorithm 2): with q the gap and Q the
// span of the empty band above the top occupied energy e_v, the segment
// [-K + iK'/2, K + iK'/2] of the parameter t (modulus r = (sqrt(Q/q) - 1) /
// (sqrt(Q/q) + 1)) maps to the upper half of a closed curve around the empty
// band by z = e_v + sqrt(qQ) (1/r + sn t) / (1/r - sn t), walked clockwise.  The
// midpoint rule takes n nodes, n from the quadrature bound
// exp(-pi^2 n / (2 log(Q/q) + 6)) <= tol (eq. rel_err_Cauchy).  Output: n
// lambdas then n weights (dz/dt times the step), interleaved re / im.
std::vector<double> cauchy_nodes(const double* e, int nv, int nc, double tol) {
  const double ev = e[nv - 1], q = e[nv] - ev, big_q = e[nv + nc - 1] - ev;
  const double ratio = std::max(big_q / q, 1.0 + 1e-12);
  int n = (int)std::ceil((2.0 * std::log(ratio) + 6.0) * std::log(1.0 / tol) / (M_PI * M_PI));
  n = std::max(4, std::min(n, CAUCHY_MAX_NODES));
  const double r = (std::sqrt(ratio) - 1.0) / (std::sqrt(ratio) + 1.0), m = r * r;
  const double kk = ellip_k(m), half = 0.5 * ellip_k(1.0 - m), sq = std::sqrt(q * big_q);
  std::vector<double> out(4 * (size_t)n);
  for (int k = 0; k < n; ++k) {
    std::complex<double> sn, cn, dn;
    jacobi_complex(-kk + 2.0 * kk * (k + 0.5) / n, half, m, sn, cn, dn);
    const std::complex<double> z = ev + sq * (1.0 / r + sn) / (1.0 / r - sn);
    const std::complex<double> w = 2.0 * sq / r * cn * dn / ((1.0 / r - sn) * (1.0 / r - sn)) * (2.0 * kk / n);
    out[2 * k] = z.real(); out[2 * k + 1] = z.imag();
    out[2 * (n + k)] = w.real(); out[2 * (n + k) + 1] = w.imag();
  }
  return out;
}

// The plane-wave list followed by every other grid vector (components in
// [-n_d/2, n_d/2)): the rows of the whole-grid Coulomb Gram, output list first.
std::vector<int32_t> full_grid_list(const int32_t* miller, int ng, int n0, int n1, int n2) {
  const long nr = (long)n0 * n1 * n2;
  std::vector<char> in(nr, 0);
  auto key = [&](int x, int y, int z) {
    return (long)((x % n0 + n0) % n0) + n0 * ((long)((y % n1 + n1) % n1) + (long)n1 * ((z % n2 + n2) % n2));
  };
  std::vector<int32_t> out(miller, miller + 3 * (size_t)ng);
  out.reserve(3 * (size_t)nr);
  for (int g = 0; g < ng; ++g) in[key(miller[3 * g], miller[3 * g + 1], miller[3 * g + 2])] = 1;
  for (int z = -(n2 / 2); z < n2 - n2 / 2; ++z)
    for (int y = -(n1 / 2); y < n1 - n1 / 2; ++y)
      for (int x = -(n0 / 2); x < n0 - n0 / 2; ++x)
        if (!in[key(x, y, z)]) {
          out.push_back(x);
          out.push_back(y);
          out.push_back(z);
        }
  return out;
}

// Workspace layout.  Offsets in bytes from the workspace base.
struct Layout {
  size_t psi_c = 0, pm = 0, mu = 0, e = 0, w = 0, s = 0, lin = 0, zt = 0, tabs = 0, t2 = 0, zg = 0,
         u = 0, l = 0, g = 0, a = 0, acopy = 0, x = 0, rres = 0, t = 0, status = 0,
         miller = 0, recip = 0, sqrtv = 0, idx = 0, total = 0;
  size_t twx = 0, twy = 0, twz = 0;  // inside tabs
  size_t w1 = 0;                     // aliases the zt region
  // frequency batch (n_omega >= 2): weights, core partials, M / M^{-1} / K, sweep scratch, S M^{-1}, H / T
  size_t wb = 0, partb = 0, mb = 0, lb = 0, qb = 0, hb = 0;
  size_t zt_bytes = 0;               // size of the zt region
  size_t t2_bytes = 0;               // size of the t2 region
  size_t part = 0, l2 = 0, lin2 = 0, q = 0;  // core partials; second -M buffer, sweep scratch, S M^-1 S scratch
  size_t pm32 = 0;                   // complex64 copy of the orbitals at the points (FP32 mode only)
  size_t bf_rows = 0, bf_pts = 0;    // bf16 hi / lo planes of the orbitals (BF16x3 mode only)
  size_t core_a = 0;                 // bf16 hi / lo planes of the empty states at the points (BF16x3 core)
  // contour-integral core: node table (lambda, weight), scaled operands, Gram pairs, running sum
  size_t cnodes = 0, cops = 0, cprod = 0, csum = 0, cpm32 = 0;
  int kx = 0, ky = 0, kz = 0, nd = 0, nsplit = 1;
};

Layout make_layout(const Problem& P, int kx, int ky, int kz, int nd) {
  Layout L;
  const size_t z = 16, el = P.m32 ? 8 : 16;
  const size_t nmu2 = (size_t)P.nmu * P.nmu;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += up(std::max<size_t>(bytes, 1)); return o; };
  L.kx = kx; L.ky = ky; L.kz = kz; L.nd = nd;
  // room for the tuned maximum of the generic core (2x default) and for the k-major core's split
  L.nsplit = std::min(P.nv, std::max(2 * core_splits(P.nmu, P.nv), 32));
  L.status = take(sizeof(StatusBlock));
  L.psi_c = P.cplx ? 0 : take((size_t)P.ns * P.nr * z);
  L.pm = take((size_t)P.ns * P.nmu * z);
  if (P.prec == P32) {
    L.pm32 = take((size_t)P.ns * P.nmu * 8);
  } else if (P.prec == PBF3) {
    L.bf_rows = take(bf3_rows_bytes(P.nr, P.nv, P.nc));
    L.bf_pts = take(bf3_points_bytes(P.nmu, P.nv, P.nc));
    if (core_bf3_fits(P.nmu, P.nc)) L.core_a = take(core_bf3_plane_bytes(P.nmu, P.nc));
  }
  if (P.core_method == 1) {
    L.cnodes = take((size_t)2 * CAUCHY_MAX_NODES * z);
    L.cops = take((size_t)CAUCHY_CHUNK * P.ns * P.nmu * z);
    L.cprod = take((size_t)2 * CAUCHY_CHUNK * nmu2 * z);
    L.csum = take(nmu2 * z);
    L.cpm32 = take((size_t)P.ns * P.nmu * 8);
  }
  // host-supplied arrays, adjacent so that one copy uploads them all
  L.mu = take((size_t)P.nmu * 4);
  L.e = take((size_t)P.ns * 8);
  L.miller = take((size_t)P.ngg * 3 * 4);
  L.recip = take(9 * 8);
  L.idx = take((size_t)(kx + ky + kz + 2 * nd + 2 * P.ngg + kx * ky + nd + 1 + P.ngg) * 4);
  L.w = take((size_t)P.nv * P.nc * 8);
  L.sqrtv = take((size_t)P.ngg * 8);
  L.twx = take((size_t)kx * P.n0 * el);
  L.twy = take((size_t)ky * P.n1 * el);
  L.twz = take((size_t)kz * P.n2 * el);
  L.tabs = L.twx;
  L.s = take(nmu2 * z);
  L.lin = take(linalg_scratch_bytes(P.nmu));
  // T2 of the separate x/y and z stages, or the fused DFT's per-z-block partial sums
  const size_t zr = (size_t)(P.zrows > 0 ? P.zrows : P.nmu);
  L.t2_bytes = std::max(zr * P.n2 * nd, (size_t)std::min(DFT_MAX_ZBLOCKS, P.n2) * zr * P.ngg) * el;
  L.t2 = take(L.t2_bytes);
  L.zg = take((size_t)P.nmu * P.ngg * el);
  L.u = take((size_t)P.ng * P.nmu * el);
  L.l = take(nmu2 * z);
  L.l2 = take(nmu2 * z);
  L.lin2 = take(linalg_scratch_bytes(P.nmu));
  L.q = take(nmu2 * z);
  L.part = take((size_t)L.nsplit * nmu2 * el);
  L.g = take(nmu2 * z);
  L.a = take(nmu2 * z);
  L.acopy = take(nmu2 * z);
  L.x = take(nmu2 * z);
  L.rres = take(nmu2 * z);
  L.t = take(nmu2 * z);
  if (P.nomega >= 2) {
    const size_t nb = (size_t)P.nomega;
    L.wb = take(nb * P.nv * P.nc * 8);
    L.partb = take(nb * nmu2 * el);
    L.mb = take(nb * nmu2 * z);
    L.lb = take(nb * linalg_scratch_bytes(P.nmu));
    L.qb = take(nb * nmu2 * z);
    L.hb = take(nb * nmu2 * z);
  }
  // big region: Zt (N_mu x Nr); once the DFT has consumed it, reused for the
  // split-K partial sums of U^H U and for U T
  const size_t zt_bytes = zr * P.nr * el;
  const size_t w1_bytes = (size_t)P.ng * P.nmu * el;
  L.zt_bytes = std::max(zt_bytes, w1_bytes);
  L.zt = take(L.zt_bytes);
  L.w1 = L.zt;
  L.total = off;
  return L;
}

template <typename T>
T* at(void* ws, size_t off) { return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off); }

isdf_status fail(isdf_handle h, isdf_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

#define HIPCHK_H(hh, expr)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(hh, ISDF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));   \
  } while (0)

#define HIPCHK(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(h, ISDF_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

#define TRY(x) do { isdf_status s_ = (x); if (s_ != ISDF_OK) return s_; } while (0)

isdf_status check_problem(isdf_handle h, const isdf_problem* pr, Problem& P) {
  if (!pr) return fail(h, ISDF_E_ARG, "problem is NULL");
  for (int d = 0; d < 3; ++d)
    if (pr->n[d] < 2 || pr->n[d] > 1024) return fail(h, ISDF_E_ARG, "grid size out of range [2, 1024]");
  if (pr->nv < 1 || pr->nc < 1) return fail(h, ISDF_E_ARG, "nv and nc must be >= 1");
  if (!(pr->pair_factor > 0.0) || !std::isfinite(pr->pair_factor)) return fail(h, ISDF_E_ARG, "pair_factor must be positive");
  if (!(pr->v_scale > 0.0) || !std::isfinite(pr->v_scale)) return fail(h, ISDF_E_ARG, "v_scale must be positive");
  if (pr->refine_steps < 0 || pr->refine_steps > 8) return fail(h, ISDF_E_ARG, "refine_steps must be in [0, 8]");
  if (pr->prec != ISDF_FP64 && pr->prec != ISDF_FP32 && pr->prec != ISDF_BF16X3) return fail(h, ISDF_E_ARG, "unknown precision");
  if (pr->is_complex != 0 && pr->is_complex != 1) return fail(h, ISDF_E_ARG, "is_complex must be 0 or 1");
  if (pr->coulomb_sum != 0 && pr->coulomb_sum != 1) return fail(h, ISDF_E_ARG, "coulomb_sum must be 0 or 1");
  if (pr->core_method != 0 && pr->core_method != 1) return fail(h, ISDF_E_ARG, "core_method must be 0 or 1");
  if (!(pr->core_tol >= 0.0 && pr->core_tol < 1e-2)) return fail(h, ISDF_E_ARG, "core_tol must be in [0, 1e-2)");
  const double* c = pr->cell;
  const double det = c[0] * (c[4] * c[8] - c[5] * c[7]) - c[1] * (c[3] * c[8] - c[5] * c[6]) + c[2] * (c[3] * c[7] - c[4] * c[6]);
  if (!(std::fabs(det) > 1e-12) || !std::isfinite(det)) return fail(h, ISDF_E_ARG, "cell is singular");
  P.n0 = pr->n[0]; P.n1 = pr->n[1]; P.n2 = pr->n[2];
  P.nr = (long)P.n0 * P.n1 * P.n2;
  P.nv = pr->nv; P.nc = pr->nc; P.ns = pr->nv + pr->nc;
  P.cplx = pr->is_complex == 1;
  P.prec = (Prec)pr->prec;
  P.m32 = P.prec != P64;
  P.f = pr->pair_factor;
  P.v_scale = pr->v_scale;
  P.refine = pr->refine_steps;
  P.full_gram = pr->coulomb_sum == 1;
  P.core_method = pr->core_method;
  P.core_tol = pr->core_tol > 0.0 ? pr->core_tol : 1e-13;
  // reciprocal basis rows b_i = 2 pi (cell^{-1})^T rows
  const double inv[9] = {(c[4] * c[8] - c[5] * c[7]) / det, -(c[1] * c[8] - c[2] * c[7]) / det, (c[1] * c[5] - c[2] * c[4]) / det,
                         -(c[3] * c[8] - c[5] * c[6]) / det, (c[0] * c[8] - c[2] * c[6]) / det, -(c[0] * c[5] - c[2] * c[3]) / det,
                         (c[3] * c[7] - c[4] * c[6]) / det, -(c[0] * c[7] - c[1] * c[6]) / det, (c[0] * c[4] - c[1] * c[3]) / det};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) P.recip[3 * i + j] = 2.0 * M_PI * inv[3 * j + i];
  return ISDF_OK;
}

isdf_status check_points(isdf_handle h, const Problem& P, const int32_t* mu, int nmu) {
  if (!mu) return fail(h, ISDF_E_ARG, "mu_idx is NULL");
  if (nmu < 1) return fail(h, ISDF_E_ARG, "n_mu must be >= 1");
  if ((long)nmu > (long)P.nv * P.nc) return fail(h, ISDF_E_ARG, "n_mu exceeds nv*nc (core would be singular)");
  if ((long)nmu > P.nr) return fail(h, ISDF_E_ARG, "n_mu exceeds Nr");
  std::vector<int32_t> s(mu, mu + nmu);
  std::sort(s.begin(), s.end());
  if (s.front() < 0 || s.back() >= P.nr) return fail(h, ISDF_E_ARG, "mu_idx out of range");
  for (int i = 1; i < nmu; ++i)
    if (s[i] == s[i - 1]) return fail(h, ISDF_E_ARG, "mu_idx has duplicate points");
  return ISDF_OK;
}

isdf_status check_energies(isdf_handle h, const Problem& P, const double* e) {
  if (!e) return fail(h, ISDF_E_ARG, "energies is NULL");
  double vmax = -INFINITY, cmin = INFINITY;
  for (int i = 0; i < P.ns; ++i) {
    if (!std::isfinite(e[i])) return fail(h, ISDF_E_ARG, "energies must be finite");
    if (i < P.nv) vmax = std::max(vmax, e[i]);
    else cmin = std::min(cmin, e[i]);
  }
  if (!(vmax < cmin)) return fail(h, ISDF_E_ARG, "no gap: max occupied energy >= min empty energy");
  return ISDF_OK;
}

isdf_status check_miller(isdf_handle h, const Problem& P, const int32_t* m, int ng) {
  if (!m) return fail(h, ISDF_E_ARG, "miller is NULL");
  if (ng < 1 || (long)ng > P.nr) return fail(h, ISDF_E_ARG, "ng must be in [1, Nr]");
  const int n[3] = {P.n0, P.n1, P.n2};
  std::vector<long> keys(ng);
  for (int g = 0; g < ng; ++g) {
    long key = 0;
    for (int d = 0; d < 3; ++d) {
      const int v = m[3 * g + d];
      if (v < -(n[d] / 2) || v >= n[d] - n[d] / 2) return fail(h, ISDF_E_ARG, "miller index out of [-n/2, n/2)");
      key = key * 2048 + (v + 1024);
    }
    keys[g] = key;
  }
  std::sort(keys.begin(), keys.end());
  for (int g = 1; g < ng; ++g)
    if (keys[g] == keys[g - 1]) return fail(h, ISDF_E_ARG, "miller list has duplicates");
  return ISDF_OK;
}

isdf_status check_ws(isdf_handle h, void* ws, size_t have, size_t need) {
  if (!ws) return fail(h, ISDF_E_WORKSPACE, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(ws) % ALIGN) return fail(h, ISDF_E_WORKSPACE, "workspace not 256-byte aligned");
  if (have < need) return fail(h, ISDF_E_WORKSPACE, "workspace too small: need " + std::to_string(need) + " bytes");
  return ISDF_OK;
}

// Stage host arrays through the handle's pinned buffer into device memory with a
// single copy: the destinations are workspace regions, packed into the pinned
// buffer at their workspace offsets relative to the first one.
struct Uploader {
  isdf_handle h;
  void* ws = nullptr;
  bool no_alloc = false;   // refuse to grow the pinned staging buffer
  struct Item { size_t off; const void* src; size_t bytes; };
  std::vector<Item> items;
  std::deque<std::vector<int32_t>> keep;   // host arrays built for this call, alive until run()
  void add(size_t off, const void* s, size_t bytes) { if (bytes) items.push_back({off, s, bytes}); }
  const int32_t* hold(std::vector<int32_t>&& v) { keep.push_back(std::move(v)); return keep.back().data(); }
  std::deque<std::vector<double>> keepd;
  const double* hold(std::vector<double>&& v) { keepd.push_back(std::move(v)); return keepd.back().data(); }
  // Items are staged in pinned memory and copied in groups: items whose workspace
  // ranges are separated by no more than alignment padding share one copy; any
  // larger gap holds other buffers and starts a new copy (so the copies never
  // write outside the items and their padding).
  isdf_status run() {
    if (items.empty()) return ISDF_OK;
    std::sort(items.begin(), items.end(), [](const Item& a, const Item& b) { return a.off < b.off; });
    struct Group { size_t lo, hi, at; };
    std::vector<Group> groups;
    for (auto& it : items) {
      if (groups.empty() || it.off > groups.back().hi + ALIGN) groups.push_back({it.off, it.off + it.bytes, 0});
      else groups.back().hi = std::max(groups.back().hi, it.off + it.bytes);
    }
    size_t total = 0;
    for (auto& g : groups) { g.at = total; total += g.hi - g.lo; }
    // the previous call's copies out of the pinned buffer must be complete
    HIPCHK(hipStreamSynchronize(h->stream));
    if (total > h->pinned_bytes && no_alloc)
      return fail(h, ISDF_E_WORKSPACE, "the host arrays (" + std::to_string(total) +
                  " bytes) do not fit the handle's pinned staging buffer (" + std::to_string(h->pinned_bytes) +
                  " bytes) and this call allocates nothing");
    if (total > h->pinned_bytes) {
      if (h->pinned) HIPCHK(hipHostFree(h->pinned));
      h->pinned = nullptr;
      h->pinned_bytes = 0;
      HIPCHK(hipHostMalloc(&h->pinned, total, hipHostMallocDefault));
      h->pinned_bytes = total;
    }
    char* base = reinterpret_cast<char*>(h->pinned);
    size_t gi = 0;
    for (auto& it : items) {
      while (it.off >= groups[gi].hi) ++gi;
      std::memcpy(base + groups[gi].at + (it.off - groups[gi].lo), it.src, it.bytes);
    }
    for (auto& g : groups)
      HIPCHK(hipMemcpyAsync(reinterpret_cast<char*>(ws) + g.lo, base + g.at, g.hi - g.lo, hipMemcpyHostToDevice,
                            h->stream));
    return ISDF_OK;
  }
};

struct Timer {
  isdf_handle h;
  bool on;
  int k = 0;
  hipEvent_t* evs = nullptr;   // events to record into (10 of them); the handle's own when null
  void mark() {
    if (on && k < 10) (void)hipEventRecord(evs ? evs[k++] : h->ev[k++], h->stream);
  }
};

// ---- shared pieces of the pipeline --------------------------------------------------------
// Launch-shape knobs (isdf_tune); defaults are what the library uses untuned.
struct Tune {
  int dft_zb = 8;          // z-planes per DFT workgroup
  int core_split_pct = 100;  // core split count, percent of the default
  int gram_split = 8;      // split-K cap of X^H X
  int wg_per_cu = 1;       // workgroups per CU of the persistent k-major kernels
  int core_stream = 0;     // first core: 0 main stream before Z, 1 side stream after Z, 2 side stream beside Z
  int side_prio = 1;       // 1: the second stream's sweep steps raise their waves' issue priority
  int dft_pipe = 1;        // 1: the warp-specialised fused DFT (single precision) where it fits
};

struct Run {
  isdf_handle h;
  Tune tune;
  Problem P;
  Layout L;
  void* ws;
  const void* psi;      // complex128 view of the orbitals (device)
  StatusBlock* sb;
  // read-only tables: workspace regions (per-call upload) or a plan's own buffer
  const int* mu = nullptr;
  const double* e = nullptr;      // energies (device)
  const int* miller = nullptr;
  const double* recip = nullptr;
  const int* idx = nullptr;       // pruned-DFT index lists
  const void* tmat = nullptr;  // T (times talpha) after the core algebra
  const void* t32 = nullptr;   // tmat in complex64 (the refinement-residual buffer), or null if not made
  int cn = 0;                  // contour nodes in the table (core_method 1)
  double talpha = 1.0;
  Prec grad_big = P64;         // adjoint: compute precision of the contractions over the grid
  bool gap_side = false;       // the energy-gap check still to enqueue, on the second stream after the fork
  hipStream_t st;
};

isdf_status prepare_psi(Run& R, const void* psi) {
  isdf_handle h = R.h;
  if (R.P.cplx) {
    R.psi = psi;
  } else {
    void* pc = at<char>(R.ws, R.L.psi_c);
    HIPCHK(widen_real((const double*)psi, pc, (long)R.P.ns * R.P.nr, R.st));
    R.psi = pc;
  }
  return ISDF_OK;
}

isdf_status stage_points(Run& R) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  HIPCHK(gather_points(R.psi, P.nr, P.ns, R.mu, P.nmu, at<char>(R.ws, R.L.pm), R.st));
  return ISDF_OK;
}

// S^T = conj(S) at the points (FP64) into the s buffer; with invert, Sw = -(S^T)^{-1} in place
isdf_status stage_s(Run& R, hipStream_t st, size_t lin, bool invert) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  void* pm = at<char>(R.ws, R.L.pm);
  void* s = at<char>(R.ws, R.L.s);
  HIPCHK(zpair(P64, P.nmu, P.nmu, P.nv, P.ns, pm, P.nmu, pm, P.nmu, false, s, P.nmu, false, st));
  if (invert) HIPCHK(sweep_inverse(P.nmu, s, at<char>(R.ws, lin), &R.sb->status, st));
  return ISDF_OK;
}

// K = S M^{-1} S in place of M^{-1} (mi), with S = conj(S^T) from the s buffer; q is scratch
isdf_status stage_smis(Run& R, void* mi, void* q, hipStream_t st) {
  isdf_handle h = R.h;
  const int n = R.P.nmu;
  const void* sk = at<char>(R.ws, R.L.s);
  GemmDesc a;  // q = M^{-1} S
  a.M = a.N = a.K = n;
  a.A = mi; a.sam = n; a.sak = 1;
  a.B = sk; a.sbk = n; a.sbn = 1; a.conjB = true;
  a.C = q; a.ldc = n;
  HIPCHK(gemm(P64, a, st));
  GemmDesc b;  // mi = S q (Hermitian: lower tiles, mirrored)
  b.M = b.N = b.K = n;
  b.A = sk; b.sam = n; b.sak = 1; b.conjA = true;
  b.B = q; b.sbk = n; b.sbn = 1;
  b.C = mi; b.ldc = n;
  b.herm = true;
  HIPCHK(gemm(P64, b, st));
  return ISDF_OK;
}

// Operands of the pair product.  FP32 mode: the orbitals at the points go to
// complex64 (the pair kernel reads the grid orbitals as they are and rounds them
// while staging).  BF16x3: both go to bf16 hi / lo planes.
isdf_status stage_z_operands(Run& R, hipStream_t st) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  if (P.prec == P64) return ISDF_OK;
  if (P.prec == PBF3) {
    HIPCHK(bf3_split_rows(R.psi, P.nr, P.nr, P.nv, P.nc, at<char>(R.ws, R.L.bf_rows), st));
    HIPCHK(bf3_split_points(at<char>(R.ws, R.L.pm), P.nmu, P.nmu, P.nv, P.nc, at<char>(R.ws, R.L.bf_pts), st));
    return ISDF_OK;
  }
  HIPCHK(convert_z(at<char>(R.ws, R.L.pm), false, at<char>(R.ws, R.L.pm32), true, (long)P.ns * P.nmu, st));
  return ISDF_OK;
}
isdf_status stage_z_operands(Run& R) { return stage_z_operands(R, R.st); }

// Z^T [mu][r] by the pair-Gram kernel (one launch).
isdf_status stage_z(Run& R) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  if (P.prec == P64) {
    HIPCHK(zpair(P64, P.nmu, (int)P.nr, P.nv, P.ns, at<char>(R.ws, R.L.pm), P.nmu, R.psi, P.nr, false,
                 at<char>(R.ws, R.L.zt), P.nr, false, R.st));
    return ISDF_OK;
  }
  if (P.prec == PBF3) {
    HIPCHK(zpair_bf3(P.nr, P.nmu, P.nv, P.nc, at<char>(R.ws, R.L.bf_rows), at<char>(R.ws, R.L.bf_pts),
                     at<char>(R.ws, R.L.zt), P.nr, R.st));
    return ISDF_OK;
  }
  HIPCHK(zpair(P32, P.nmu, (int)P.nr, P.nv, P.ns, at<char>(R.ws, R.L.pm32), P.nmu, R.psi, P.nr, true,
               at<char>(R.ws, R.L.zt), P.nr, true, R.st, R.tune.wg_per_cu));
  return ISDF_OK;
}

DftPlan make_plan(Run& R) {
  const Problem& P = R.P;
  const Layout& L = R.L;
  DftPlan p;
  p.n0 = P.n0; p.n1 = P.n1; p.n2 = P.n2; p.nmu = P.nmu; p.ng = P.ngg;
  p.kx = L.kx; p.ky = L.ky; p.nd = L.nd; p.kz = L.kz;
  p.zb = R.tune.dft_zb;
  p.pipe = R.tune.dft_pipe;
  p.twx = at<char>(R.ws, L.twx);
  p.twy = at<char>(R.ws, L.twy);
  p.twz = at<char>(R.ws, L.twz);
  const int* ib = R.idx;
  // idx block: xl[kx] yl[ky] zl[kz] d_ax[nd] d_by[nd] g_d[ng] g_cz[ng] dmap[kx][ky] gd_off[nd + 1] gd_list[ng]
  p.d_ax = ib + L.kx + L.ky + L.kz;
  p.d_by = p.d_ax + L.nd;
  p.g_d = p.d_by + L.nd;
  p.g_cz = p.g_d + P.ngg;
  p.dmap = p.g_cz + P.ngg;
  p.gd_off = p.dmap + L.kx * L.ky;
  p.gd_list = p.gd_off + L.nd + 1;
  return p;
}

// The pruned DFT of p.nmu rows zt[mu][r] onto the plane-wave list (times scale[g] if
// given): the fused pass when the shape fits, else the x/y and z kernels.  t2 is the
// scratch of either (t2_bytes).
isdf_status dft_apply(Run& R, const DftPlan& p, const void* zt, void* t2, size_t t2_bytes, void* zg,
                      const double* scale) {
  isdf_handle h = R.h;
  const Prec cp = R.P.prec == P64 ? P64 : P32;
  if (dft_fused_fits(cp, p)) {
    const hipError_t e = dft_fused(cp, p, zt, t2, t2_bytes, zg, scale, R.st);
    if (e == hipSuccess) return ISDF_OK;
    if (e != hipErrorNotSupported) HIPCHK(e);
  }
  HIPCHK(dft_xy(cp, p, zt, t2, R.st));
  HIPCHK(dft_z(cp, p, t2, zg, scale, R.st));
  return ISDF_OK;
}

// Unitary DFT of the N_mu rows of Z^T on the plane-wave list.  With scaled = true the
// result is X^T = (V^{1/2} F Z)^T, [mu][g] in the zg buffer.
isdf_status dft_tables(Run& R, hipStream_t st) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const int* ib = R.idx;
  HIPCHK(coulomb_sqrt(R.miller, P.ngg, R.recip, P.v_scale, at<double>(R.ws, L.sqrtv), st));
  HIPCHK(dft_twiddles(ib, L.kx, P.n0, P.m32, at<char>(R.ws, L.twx), st));
  HIPCHK(dft_twiddles(ib + L.kx, L.ky, P.n1, P.m32, at<char>(R.ws, L.twy), st));
  HIPCHK(dft_twiddles(ib + L.kx + L.ky, L.kz, P.n2, P.m32, at<char>(R.ws, L.twz), st));
  return ISDF_OK;
}
isdf_status dft_tables(Run& R) { return dft_tables(R, R.st); }

// tables: false when the caller has already enqueued dft_tables (and ordered them before this)
isdf_status stage_dft(Run& R, bool scaled, bool tables = true) {
  const Layout& L = R.L;
  if (tables) TRY(dft_tables(R));
  DftPlan p = make_plan(R);
  const double* scale = scaled ? at<double>(R.ws, L.sqrtv) : nullptr;
  return dft_apply(R, p, at<char>(R.ws, L.zt), at<char>(R.ws, L.t2), L.t2_bytes, at<char>(R.ws, L.zg), scale);
}

// U = X S^{-1} (stage entry only): U(g, nu) = sum_mu Xt[mu][g] S^{-1}(mu, nu), S^{-1}(mu, nu) = -Sw[nu][mu]
isdf_status stage_u(Run& R) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const Prec cp = P.prec == P64 ? P64 : P32;
  GemmDesc d;
  d.M = P.ng; d.N = P.nmu; d.K = P.nmu;
  d.A = at<char>(R.ws, L.zg); d.sam = 1; d.sak = P.ngg; d.a32 = P.m32;
  d.B = at<char>(R.ws, L.s); d.sbk = 1; d.sbn = P.nmu;
  d.C = at<char>(R.ws, L.u); d.ldc = P.nmu; d.c32 = P.m32;
  d.alpha = -1.0;
  HIPCHK(gemm(cp, d, R.st));
  return ISDF_OK;
}

// An NG x N_mu plane-wave basis B(g, mu) = base[g * sg + mu * smu] in mode precision:
// X (from X^T, sg = 1, smu = NG) or U (row-major, sg = N_mu, smu = 1).
struct Basis {
  const void* base;
  long sg, smu;
};

// G = B^H B (Hermitian, split-K over the plane waves)
isdf_status stage_gram(Run& R, const Basis& b) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Prec cp = P.prec == P64 ? P64 : P32;
  // Single precision with X^T stored [point][plane wave]: a [plane wave][point] copy in
  // the Z^T region (free once the DFT has run) makes both operands of G = X^H X k-major,
  // for the persistent engine; the rest of the region holds its split-tail slices.
  char* xg = at<char>(R.ws, R.L.zt);
  const size_t xbytes = up((size_t)P.ngg * P.nmu * 8);
  if (P.m32 && b.sg == 1 && b.smu >= P.ngg && R.L.zt_bytes >= xbytes &&
      gemm32_fits(P.nmu, P.nmu, P.ngg, xg, P.nmu, xg, P.nmu)) {
    HIPCHK(transpose_c32(P.nmu, P.ngg, b.base, b.smu, xg, R.st));
    HIPCHK(gemm32_kmajor(P.nmu, P.nmu, P.ngg, xg, P.nmu, true, xg, P.nmu, false, at<char>(R.ws, R.L.g), P.nmu, true,
                         1.0, R.st, R.tune.wg_per_cu, xg + xbytes, R.L.zt_bytes - xbytes, 0.0));
    return ISDF_OK;
  }
  GemmDesc d;
  d.M = d.N = P.nmu; d.K = P.ngg;   // over the Gram's plane waves (the list, or the whole grid)
  d.A = b.base; d.sam = b.smu; d.sak = b.sg; d.conjA = true; d.a32 = P.m32;
  d.B = b.base; d.sbk = b.sg; d.sbn = b.smu; d.b32 = P.m32;
  d.C = at<char>(R.ws, R.L.g); d.ldc = P.nmu;
  d.herm = true;
  d.split_ws = at<char>(R.ws, R.L.zt);    // Z^T region, free once the DFT has run
  d.max_split = R.tune.gram_split;
  d.split_ws_bytes = R.L.zt_bytes;
  HIPCHK(gemm(cp, d, R.st));
  return ISDF_OK;
}

// core M at one frequency: written to m_out (if given) and/or -M to negm
// Core by the contour integral (Algorithm 2), static: chunks of nodes, each a
// scaling pass, two batched Gram products and a fixed-order Hadamard accumulation.
isdf_status stage_core_cauchy(Run& R, void* m_out, void* negm, hipStream_t st) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const Prec cp = P.prec == P64 ? P64 : P32;
  const int n = P.nmu, nv = P.nv, ns = P.ns;
  const long n2 = (long)n * n;
  char* pm = at<char>(R.ws, L.pm);
  char* ops = at<char>(R.ws, L.cops);
  char* av = at<char>(R.ws, L.cprod);
  char* ac = av + (size_t)CAUCHY_CHUNK * n2 * 16;
  const char* lam = at<char>(R.ws, L.cnodes);
  const char* wts = lam + (size_t)R.cn * 16;
  HIPCHK(zero_fill(at<char>(R.ws, L.csum), (size_t)n2 * 16, st));
  // single precision on full tiles: the Gram pairs on the k-major engine, complex64 operands and products
  char* pm32 = at<char>(R.ws, L.cpm32);
  const size_t opsz = (size_t)ns * n * 8;   // one node's complex64 operands
  const bool km = cp == P32 && opsz % 16 == 0 && ((size_t)n2 * 8) % 16 == 0 &&
                  gemm32_fits(n, n, nv, pm32, n, ops, n) &&
                  gemm32_fits(n, n, P.nc, pm32 + (size_t)nv * n * 8, n, ops + (size_t)nv * n * 8, n);
  if (km) {
    HIPCHK(convert_z(pm, false, pm32, true, (long)ns * n, st));
    char* av32 = av;
    char* ac32 = av + (size_t)CAUCHY_CHUNK * n2 * 8;
    for (int k0 = 0; k0 < R.cn; k0 += CAUCHY_CHUNK) {
      const int kc = std::min(CAUCHY_CHUNK, R.cn - k0);
      HIPCHK(cauchy_scale(pm, R.e, lam, n, nv, ns, k0, kc, ops, true, st));
      for (int kk = 0; kk < kc; ++kk) {
        char* o = ops + kk * opsz;
        HIPCHK(gemm32_kmajor(n, n, nv, pm32, n, true, o, n, false, av32 + (size_t)kk * n2 * 8, n, false, 1.0, st,
                             R.tune.wg_per_cu));
        HIPCHK(gemm32_kmajor(n, n, P.nc, pm32 + (size_t)nv * n * 8, n, false, o + (size_t)nv * n * 8, n, false,
                             ac32 + (size_t)kk * n2 * 8, n, false, 1.0, st, R.tune.wg_per_cu));
      }
      HIPCHK(cauchy_accum(av32, ac32, true, wts, k0, kc, n, at<char>(R.ws, L.csum), st));
    }
    HIPCHK(cauchy_finish(at<char>(R.ws, L.csum), n, P.f, m_out, negm, st));
    return ISDF_OK;
  }
  for (int k0 = 0; k0 < R.cn; k0 += CAUCHY_CHUNK) {
    const int kc = std::min(CAUCHY_CHUNK, R.cn - k0);
    HIPCHK(cauchy_scale(pm, R.e, lam, n, nv, ns, k0, kc, ops, false, st));
    GemmDesc a;   // Av_k(mu, nu) = sum_i conj(psi_i(mu)) ops_k[i][nu]
    a.M = a.N = n; a.K = nv;
    a.A = pm; a.sam = 1; a.sak = n; a.conjA = true;
    a.B = ops; a.sbk = n; a.sbn = 1;
    a.C = av; a.ldc = n;
    a.batch = kc; a.bsa = 0; a.bsb = (long)ns * n; a.bsc = n2;
    HIPCHK(gemm(cp, a, st));
    GemmDesc c = a;   // Ac_k(mu, nu) = sum_j psi_j(mu) ops_k[j][nu] (ops holds conj(psi_j) / (lambda - eps_j))
    c.K = P.nc;
    c.A = pm + (size_t)nv * n * 16; c.conjA = false;
    c.B = ops + (size_t)nv * n * 16;
    c.C = ac;
    HIPCHK(gemm(cp, c, st));
    HIPCHK(cauchy_accum(av, ac, false, wts, k0, kc, n, at<char>(R.ws, L.csum), st));
  }
  HIPCHK(cauchy_finish(at<char>(R.ws, L.csum), n, P.f, m_out, negm, st));
  return ISDF_OK;
}

isdf_status stage_core(Run& R, double omega, void* m_out, void* negm, hipStream_t st) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Prec cp = P.prec == P64 ? P64 : P32;
  if (P.core_method == 1) {
    if (omega != 0.0) return fail(h, ISDF_E_UNSUPPORTED, "the contour-integral core is static (omega = 0)");
    return stage_core_cauchy(R, m_out, negm, st);
  }
  double* w = at<double>(R.ws, R.L.w);
  HIPCHK(pair_weights(R.e, P.nv, P.nc, omega, w, st));
  void* part = at<char>(R.ws, R.L.part);
  if (P.prec == PBF3 && R.L.core_a) {
    void* planes = at<char>(R.ws, R.L.core_a);
    const int ns = core32_splits(P.nmu, P.nv, R.L.nsplit);
    HIPCHK(core_bf3_split(P.nmu, P.nv, P.nc, at<char>(R.ws, R.L.pm), planes, st));
    HIPCHK(core_bf3_partial(P.nmu, P.nv, P.nc, at<char>(R.ws, R.L.pm), planes, w, part, ns, st));
    HIPCHK(core_reduce(cp, P.nmu, part, ns, P.f, m_out, negm, st));
    return ISDF_OK;
  }
  if (cp == P32 && core32_fits(P.nmu, P.nc)) {
    const int ns = core32_splits(P.nmu, P.nv, R.L.nsplit);
    HIPCHK(core32_partial(P.nmu, P.nv, P.nc, at<char>(R.ws, R.L.pm), w, part, ns, st));
    HIPCHK(core_reduce(cp, P.nmu, part, ns, P.f, m_out, negm, st));
    return ISDF_OK;
  }
  const int ns = std::max(1, std::min(R.L.nsplit, core_splits(P.nmu, P.nv) * R.tune.core_split_pct / 100));
  HIPCHK(core_partial(cp, P.nmu, P.nv, P.nc, at<char>(R.ws, R.L.pm), P.nmu, w, part, ns, st));
  HIPCHK(core_reduce(cp, P.nmu, part, ns, P.f, m_out, negm, st));
  return ISDF_OK;
}

// SMW core, all FP64: H = G - K (Hermitian positive definite), T = H^{-1} = -sweep(H),
// optional Newton refinement T <- T + T (I - H T) with residuals ||I - H T||_F / sqrt(n).
// With B the plane-wave basis of stage_gram, eps~^{-1} = I - B T B^H.
//   B = U (= X S^{-1}):  G = U^H U, K = M^{-1}
//   B = X (= V^{1/2} F Z): G = X^H X, K = S M^{-1} S   (S^{-1} never formed)
// `used` (optional) is recorded once K has been read.
// FP64 Newton refinement T <- T + T (I - H T) of an inverse, from Hc (a copy of H)
// and T0 = tneg * (first inverse), with residuals ||I - H T_k||_F^2 in the status
// block; sets R.tmat / R.talpha.
isdf_status refine_inverse(Run& R, const void* Hc, const void* Tfirst, double tneg) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const int n = P.nmu;
  const long n2 = (long)n * n;
  void* T = at<char>(R.ws, L.t);
  void* T2 = at<char>(R.ws, L.x);
  void* Rr = at<char>(R.ws, L.rres);
  HIPCHK(scale_z(Tfirst, T, n2, tneg, R.st));
  for (int k = 0; k <= P.refine; ++k) {
    GemmDesc r;  // Rr = I - H T
    r.M = r.N = r.K = n;
    r.A = Hc; r.sam = n; r.sak = 1;
    r.B = T; r.sbk = n; r.sbn = 1;
    r.C = Rr; r.ldc = n; r.alpha = -1.0; r.diag_add = 1.0;
    HIPCHK(gemm(P64, r, R.st));
    HIPCHK(frob2(Rr, n2, R.sb->partial, &R.sb->res[k], R.st));
    if (k == P.refine) break;
    HIPCHK(convert_z(T, false, T2, false, n2, R.st));
    GemmDesc c;  // T2 = T + T Rr: the correction is ||Rr|| times smaller than T, so its
    c.M = c.N = c.K = n;   // product runs on FP32 MFMA (FP64 storage and accumulation into T)
    c.A = T; c.sam = n; c.sak = 1;
    c.B = Rr; c.sbk = n; c.sbn = 1;
    c.C = T2; c.ldc = n; c.beta = 1.0;
    HIPCHK(gemm(P32, c, R.st));
    std::swap(T, T2);
  }
  R.tmat = T;
  R.t32 = nullptr;
  R.talpha = 1.0;
  return ISDF_OK;
}

isdf_status stage_core_algebra(Run& R, void* Mi, hipEvent_t used) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const int n = P.nmu;
  const long n2 = (long)n * n;
  void* H = at<char>(R.ws, L.a);
  // H = G - K, with ||H||_F^2 and its smallest diagonal entry for the status block
  // (and the sweep's first pivot block inverse, in the same launch)
  HIPCHK(form_h(at<char>(R.ws, L.g), Mi, H, n, R.sb->partial, &R.sb->h2, &R.sb->min_pivot, R.st,
                at<char>(R.ws, L.lin), &R.sb->status));
  if (used) HIPCHK(hipEventRecord(used, R.st));
  if (P.refine > 0) HIPCHK(convert_z(H, false, at<char>(R.ws, L.acopy), false, n2, R.st));
  HIPCHK(sweep_inverse(n, H, at<char>(R.ws, L.lin), &R.sb->status, R.st, 1, true, true));   // -T
  // ||T||_F^2, and without refinement in single precision T's complex64 copy for the
  // output products in the same pass (the refinement-residual buffer is free then)
  void* t32 = (P.m32 && P.refine == 0) ? at<char>(R.ws, L.rres) : nullptr;
  HIPCHK(frob2(H, n2, R.sb->partial, &R.sb->t2, R.st, t32));
  R.tmat = H;
  R.t32 = t32;
  R.talpha = -1.0;
  if (P.refine == 0) return ISDF_OK;
  return refine_inverse(R, at<char>(R.ws, L.acopy), H, -1.0);
}

isdf_status stage_out(Run& R, const Basis& b, void* out, Timer& tm) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const Prec cp = P.prec == P64 ? P64 : P32;
  if (P.m32 && b.sg == 1 && b.smu >= P.ng && gemm32_fits(P.nmu, P.ng, P.nmu, b.base, b.smu, b.base, b.smu) &&
      gemm32_fits(P.ng, P.ng, P.nmu, at<char>(R.ws, L.w1), P.ng, b.base, b.smu)) {
    // Mixed path with the basis stored [point][plane wave] (X^T): both products
    // have k-major operands.  W^T = talpha T^T X^T, then eps~^{-1} = I - W X^H.
    // T goes to complex64 in the refinement-residual buffer (free by now).
    void* t32 = at<char>(R.ws, L.rres);
    void* wt = at<char>(R.ws, L.w1);
    if (R.t32 != t32) HIPCHK(convert_z(R.tmat, false, t32, true, (long)P.nmu * P.nmu, R.st));
    // the t2 region (DFT scratch, consumed by now) holds the K slices of the split tails
    void* tail = at<char>(R.ws, L.t2);
    HIPCHK(gemm32_kmajor(P.nmu, P.ng, P.nmu, t32, P.nmu, false, b.base, b.smu, false, wt, P.ng, false,
                         R.talpha, R.st, R.tune.wg_per_cu, tail, L.t2_bytes));
    tm.mark();
    HIPCHK(gemm32_kmajor(P.ng, P.ng, P.nmu, wt, P.ng, false, b.base, b.smu, true, out, P.ng, true, -1.0, R.st,
                         R.tune.wg_per_cu, tail, L.t2_bytes));
    return ISDF_OK;
  }
  GemmDesc d;  // W1 = B T
  d.M = P.ng; d.N = P.nmu; d.K = P.nmu;
  d.A = b.base; d.sam = b.sg; d.sak = b.smu; d.a32 = P.m32;
  d.B = R.tmat; d.sbk = P.nmu; d.sbn = 1;
  d.C = at<char>(R.ws, L.w1); d.ldc = P.nmu; d.c32 = P.m32;
  d.alpha = R.talpha;
  HIPCHK(gemm(cp, d, R.st));
  tm.mark();
  GemmDesc o;  // eps~^{-1} = I - W1 B^H
  o.M = o.N = P.ng; o.K = P.nmu;
  o.A = at<char>(R.ws, L.w1); o.sam = P.nmu; o.sak = 1; o.a32 = P.m32;
  o.B = b.base; o.sbk = b.smu; o.sbn = b.sg; o.conjB = true; o.b32 = P.m32;
  o.C = out; o.ldc = P.ng;
  o.alpha = -1.0; o.diag_add = 1.0; o.herm = true;
  HIPCHK(gemm(cp, o, R.st));
  return ISDF_OK;
}

isdf_status begin(isdf_handle h, const isdf_problem* prob, Problem& P, int nmu, int ng, int nomega) {
  isdf_status s = check_problem(h, prob, P);
  if (s != ISDF_OK) return s;
  P.nmu = nmu;
  P.ng = ng;
  P.ngg = P.full_gram ? (int)P.nr : ng;
  P.nomega = nomega;
  return ISDF_OK;
}

// Device status bits: 1 = a matrix that must be Hermitian positive definite is
// not; 2 = the energies have no gap (or are not finite), found on the device.
enum { ST_NOT_PD = 1, ST_NO_GAP = 2 };

isdf_status report_status(isdf_handle h, const StatusBlock& hs, const Problem& P, isdf_report* rep) {
  if (rep) {
    rep->min_pivot = hs.min_pivot;
    rep->cond_est = std::sqrt(hs.h2 * hs.t2);
    rep->n_refine_reported = P.refine > 0 ? P.refine + 1 : 0;
    for (int k = 0; k < 9; ++k)
      rep->refine_residual[k] = k < rep->n_refine_reported ? std::sqrt(hs.res[k] / (double)P.nmu) : 0.0;
  }
  if (hs.status & ST_NO_GAP) return fail(h, ISDF_E_ARG, "no gap: max occupied energy >= min empty energy (or energies not finite)");
  if (hs.status & ST_NOT_PD) return fail(h, ISDF_E_NOT_PD, "a matrix that must be Hermitian positive definite is not (S = C C^H, -M or X^H X - S M^{-1} S)");
  h->err.clear();
  return ISDF_OK;
}

isdf_status finish(Run& R, isdf_report* rep, Timer& tm) {
  isdf_handle h = R.h;
  StatusBlock hs;
  HIPCHK(hipMemcpyAsync(&hs, R.sb, offsetof(StatusBlock, partial), hipMemcpyDeviceToHost, R.st));
  HIPCHK(hipStreamSynchronize(R.st));
  if (rep) {
    if (tm.on) {
      for (int k = 0; k < 8; ++k) rep->stage_ms[k] = 0.0;
      for (int k = 0; k + 1 < tm.k && k < 8; ++k) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev[k], h->ev[k + 1]));
        rep->stage_ms[k] = ms;
      }
    }
  }
  return report_status(h, hs, R.P, rep);
}

isdf_status setup_common(Run& R, isdf_handle h, const isdf_problem* prob, const void* psi,
                         const int32_t* mu_idx, int n_mu, const int32_t* miller, int ng,
                         const double* energies, int nomega, void* ws, size_t ws_bytes, Uploader& up_,
                         DftIndex& ix, std::vector<int>& idxbuf, bool grad = false) {
  if (!h) return ISDF_E_ARG;
  isdf_status s = begin(h, prob, R.P, n_mu, ng, nomega);
  if (s != ISDF_OK) return s;
  if (grad) R.P.zrows = grad_chunk(R.P);
  if (!psi) return fail(h, ISDF_E_ARG, "psi is NULL");
  s = check_points(h, R.P, mu_idx, n_mu);
  if (s != ISDF_OK) return s;
  if (miller) {
    s = check_miller(h, R.P, miller, ng);
    if (s != ISDF_OK) return s;
    // the Gram's plane waves: the list itself, or the list followed by the rest of the grid
    if (R.P.full_gram) miller = up_.hold(full_grid_list(miller, ng, R.P.n0, R.P.n1, R.P.n2));
    ix = dft_index(miller, R.P.ngg);
    if (!dft_supported(R.P.n0, R.P.n1, R.P.n2, (int)ix.xl.size(), (int)ix.yl.size(), R.P.prec == P64 ? P64 : P32))
      return fail(h, ISDF_E_UNSUPPORTED, "grid axis above 64 points: the DFT keeps an x-y slab in LDS and a z-line per wave");
  } else {
    R.P.ngg = ng;   // no Gram in this call
    ix.xl = ix.yl = ix.zl = {0};
    ix.d_ax = ix.d_by = {0};
    ix.dmap = {-1};
  }
  if (energies) {
    s = check_energies(h, R.P, energies);
    if (s != ISDF_OK) return s;
  }
  R.L = make_layout(R.P, (int)ix.xl.size(), (int)ix.yl.size(), (int)ix.zl.size(), (int)ix.d_ax.size());
  s = check_ws(h, ws, ws_bytes, R.L.total);
  if (s != ISDF_OK) return s;
  R.h = h;
  R.ws = ws;
  R.st = h->stream;
  R.sb = at<StatusBlock>(ws, R.L.status);
  R.mu = at<int>(ws, R.L.mu);
  R.e = at<double>(ws, R.L.e);
  R.miller = at<int>(ws, R.L.miller);
  R.recip = at<double>(ws, R.L.recip);
  R.idx = at<int>(ws, R.L.idx);
  up_.h = h;
  up_.ws = ws;
  up_.add(R.L.mu, mu_idx, (size_t)n_mu * 4);
  if (energies) up_.add(R.L.e, energies, (size_t)R.P.ns * 8);
  if (energies && R.P.core_method == 1) {
    std::vector<double> nodes = cauchy_nodes(energies, R.P.nv, R.P.nc, R.P.core_tol);
    R.cn = (int)(nodes.size() / 4);
    const size_t bytes = nodes.size() * 8;
    up_.add(R.L.cnodes, up_.hold(std::move(nodes)), bytes);
  }
  if (miller) {
    up_.add(R.L.miller, miller, (size_t)R.P.ngg * 12);
    idxbuf.clear();
    for (auto* v : {&ix.xl, &ix.yl, &ix.zl, &ix.d_ax, &ix.d_by, &ix.g_d, &ix.g_cz, &ix.dmap, &ix.gd_off, &ix.gd_list})
      idxbuf.insert(idxbuf.end(), v->begin(), v->end());
    up_.add(R.L.idx, idxbuf.data(), idxbuf.size() * 4);
    up_.add(R.L.recip, R.P.recip, 9 * 8);
  }
  return ISDF_OK;
}

isdf_status clear_status(Run& R) {
  isdf_handle h = R.h;
  HIPCHK(zero_fill(R.sb, offsetof(StatusBlock, partial), R.st));
  return ISDF_OK;
}


// Enqueue the whole path on the handle's stream (and its second stream, joined
// back before returning).  No host synchronisation; the status block collects
// error bits.
// Frequency batch (n_omega >= 2).  X, X^H X and S are frequency independent and
// formed once; every frequency-dependent step runs as one batched launch over
// all frequencies: the weights and cores M(omega) (this stream, ahead of Z), the
// sweeps to M(omega)^{-1} and K(omega) = S M^{-1} S (second stream, overlapping
// Z and the DFT), H(omega) = X^H X - K(omega) and its sweep (this stream).  Only
// the two output products run per frequency.
isdf_status enqueue_eps_inv_batched(Run& R, const double* omega, int nw, void* eps_inv, Timer& tm) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const Prec cp = P.prec == P64 ? P64 : P32;
  const int n = P.nmu, ng = P.ng;
  const long n2 = (long)n * n;
  hipStream_t side = h->side;
  HIPCHK(hipEventRecord(h->fork, R.st));
  HIPCHK(hipStreamWaitEvent(side, h->fork, 0));
  if (R.gap_side) HIPCHK(check_gap(R.e, P.nv, P.nc, &R.sb->status, ST_NO_GAP, side));
  TRY(stage_s(R, side, L.lin2, false));
  // the pair kernel's operand pass (streaming, memory-bound) beside the first core
  TRY(stage_z_operands(R, side));
  HIPCHK(hipEventRecord(h->zops, side));
  double* wb = at<double>(R.ws, L.wb);
  for (int k = 0; k < nw; ++k)
    HIPCHK(pair_weights(R.e, P.nv, P.nc, omega[k], wb + (long)k * P.nv * P.nc, R.st));
  void* mb = at<char>(R.ws, L.mb);
  if (P.prec == PBF3 && L.core_a) {
    HIPCHK(core_bf3_split(n, P.nv, P.nc, at<char>(R.ws, L.pm), at<char>(R.ws, L.core_a), R.st));
    HIPCHK(core_bf3_partial(n, P.nv, P.nc, at<char>(R.ws, L.pm), at<char>(R.ws, L.core_a), wb,
                            at<char>(R.ws, L.partb), 1, R.st, nw));
  } else if (cp == P32 && core32_fits(n, P.nc))
    HIPCHK(core32_partial(n, P.nv, P.nc, at<char>(R.ws, L.pm), wb, at<char>(R.ws, L.partb), 1, R.st, nw));
  else
    HIPCHK(core_partial(cp, n, P.nv, P.nc, at<char>(R.ws, L.pm), n, wb, at<char>(R.ws, L.partb), 1, R.st, nw));
  HIPCHK(core_reduce(cp, n, at<char>(R.ws, L.partb), 1, P.f, nullptr, mb, R.st, nw));      // -M(omega)
  HIPCHK(hipEventRecord(h->core0, R.st));
  // the pair kernel goes into the main stream ahead of the side stream's sweep launches
  HIPCHK(hipStreamWaitEvent(R.st, h->zops, 0));
  tm.mark();
  TRY(stage_z(R));
  HIPCHK(hipStreamWaitEvent(side, h->core0, 0));
  HIPCHK(sweep_inverse(n, mb, at<char>(R.ws, L.lb), &R.sb->status, side, nw, R.tune.side_prio != 0));  // M(omega)^{-1}
  {
    const void* sk = at<char>(R.ws, L.s);   // S^T = conj(S)
    void* qb = at<char>(R.ws, L.qb);
    GemmDesc a;  // q = M^{-1} S
    a.M = a.N = a.K = n;
    a.A = mb; a.sam = n; a.sak = 1;
    a.B = sk; a.sbk = n; a.sbn = 1; a.conjB = true;
    a.C = qb; a.ldc = n;
    a.batch = nw; a.bsa = n2; a.bsb = 0; a.bsc = n2;
    HIPCHK(gemm(P64, a, side));
    GemmDesc b;  // K = S q, over M^{-1} (Hermitian: lower tiles, mirrored)
    b.M = b.N = b.K = n;
    b.A = sk; b.sam = n; b.sak = 1; b.conjA = true;
    b.B = qb; b.sbk = n; b.sbn = 1;
    b.C = mb; b.ldc = n;
    b.herm = true;
    b.batch = nw; b.bsa = 0; b.bsb = n2; b.bsc = n2;
    HIPCHK(gemm(P64, b, side));
  }
  HIPCHK(hipEventRecord(h->m_ready[0], side));
  tm.mark();
  TRY(stage_dft(R, true));
  tm.mark();
  const Basis xb{at<char>(R.ws, L.zg), 1, (long)P.ngg};
  TRY(stage_gram(R, xb));
  tm.mark();
  HIPCHK(hipStreamWaitEvent(R.st, h->m_ready[0], 0));
  void* hb = at<char>(R.ws, L.hb);
  HIPCHK(sub_bcast(at<char>(R.ws, L.g), mb, hb, n2, nw, R.st));                          // H(omega)
  HIPCHK(diag_min(hb, n, &R.sb->min_pivot, R.st, nw));
  char* hlast = at<char>(R.ws, L.hb) + (size_t)(nw - 1) * n2 * 16;
  HIPCHK(frob2(hlast, n2, R.sb->partial, &R.sb->h2, R.st));
  HIPCHK(sweep_inverse(n, hb, at<char>(R.ws, L.lb), &R.sb->status, R.st, nw));            // -T(omega)
  HIPCHK(frob2(hlast, n2, R.sb->partial, &R.sb->t2, R.st));
  for (int k = 0; k < nw; ++k) {
    Timer dummy{h, false};
    Timer& t = (k == nw - 1) ? tm : dummy;
    char* tk = at<char>(R.ws, L.hb) + (size_t)k * n2 * 16;
    R.tmat = tk;
    R.t32 = nullptr;
    R.talpha = -1.0;
    if (P.refine > 0) {
      void* hc = at<char>(R.ws, L.acopy);
      HIPCHK(sub_bcast(at<char>(R.ws, L.g), at<char>(R.ws, L.mb) + (size_t)k * n2 * 16, hc, n2, 1, R.st));
      TRY(refine_inverse(R, hc, tk, -1.0));
    }
    t.mark();
    void* out = reinterpret_cast<char*>(eps_inv) + (size_t)k * ng * ng * 16;
    TRY(stage_out(R, xb, out, t));
    t.mark();
  }
  HIPCHK(hipEventRecord(h->join, side));
  HIPCHK(hipStreamWaitEvent(R.st, h->join, 0));
  return ISDF_OK;
}

isdf_status enqueue_eps_inv(Run& R, const void* psi, const double* omega, int n_omega, void* eps_inv,
                            Timer& tm) {
  isdf_handle h = R.h;
  const int ng = R.P.ng;
  TRY(prepare_psi(R, psi));
  TRY(stage_points(R));
  if (n_omega >= 2 && R.P.nomega >= 2) return enqueue_eps_inv_batched(R, omega, n_omega, eps_inv, tm);
  // Fork: the side stream forms S = C C^H and, per frequency, M^{-1} and
  // K = S M^{-1} S (double-buffered), while this stream runs Z, the DFT to
  // X = V^{1/2} F Z and X^H X.  Then eps~^{-1} = I - X (X^H X - K)^{-1} X^H, which
  // equals eq. epsilon_with_SMW with U = X S^{-1}; S^{-1} is never formed.
  // The first core M (a compute-bound kernel that would otherwise hold the CUs
  // the pair kernel starts on) runs on this stream ahead of Z; the later ones,
  // and every latency-bound sweep step, run on the side stream.  Work is enqueued
  // frequency by frequency so that every stream wait is enqueued after the event
  // record it waits for.
  hipStream_t side = h->side;
  HIPCHK(hipEventRecord(h->fork, R.st));
  HIPCHK(hipStreamWaitEvent(side, h->fork, 0));
  // the energy-gap check only sets a status bit read at the end: off the critical path
  if (R.gap_side) HIPCHK(check_gap(R.e, R.P.nv, R.P.nc, &R.sb->status, ST_NO_GAP, side));
  const int nw = std::max(n_omega, 1);
  void* mbuf[2] = {at<char>(R.ws, R.L.l), at<char>(R.ws, R.L.l2)};
  // core_stream 1: the first core waits for Z on the side stream instead, beside the DFT;
  // 2: on the side stream right after the operand pass, beside Z
  const bool core_side = R.tune.core_stream != 0;
  const bool core_beside_z = R.tune.core_stream == 2;
  // side_tail: M^{-1} and K = S M^{-1} S of frequency k on the side stream, once
  // its core M is in mbuf
  auto side_tail = [&](int k) -> isdf_status {
    HIPCHK(sweep_inverse(R.P.nmu, mbuf[k & 1], at<char>(R.ws, R.L.lin2), &R.sb->status, side, 1,
                         R.tune.side_prio != 0));                                                // M^{-1}
    TRY(stage_smis(R, mbuf[k & 1], at<char>(R.ws, R.L.q), side));                                 // S M^{-1} S
    HIPCHK(hipEventRecord(h->m_ready[k & 1], side));
    return ISDF_OK;
  };
  auto side_core = [&](int k) -> isdf_status {
    if (k >= 2) HIPCHK(hipStreamWaitEvent(side, h->m_used[k & 1], 0));
    if (k == 0 && !core_beside_z) HIPCHK(hipStreamWaitEvent(side, h->zdone, 0));
    TRY(stage_core(R, n_omega ? omega[k] : 0.0, nullptr, mbuf[k & 1], side));
    return side_tail(k);
  };
  TRY(stage_s(R, side, R.L.lin2, false));
  // the pair kernel's operand pass (streaming, memory-bound) beside the first core
  TRY(stage_z_operands(R, side));
  HIPCHK(hipEventRecord(h->zops, side));
  // the DFT's tables too (a few small launches that would otherwise sit between Z and the DFT)
  TRY(dft_tables(R, side));
  HIPCHK(hipEventRecord(h->tabs, side));
  if (!core_side) {
    TRY(stage_core(R, n_omega ? omega[0] : 0.0, nullptr, mbuf[0], R.st));
    HIPCHK(hipEventRecord(h->core0, R.st));
  }
  // The pair kernel is enqueued before the side stream's many small sweep
  // launches, so that host-side launch latency never holds it back.
  HIPCHK(hipStreamWaitEvent(R.st, h->zops, 0));
  tm.mark();
  TRY(stage_z(R));
  if (core_side) HIPCHK(hipEventRecord(h->zdone, R.st));
  if (!core_side) {
    HIPCHK(hipStreamWaitEvent(side, h->core0, 0));
    TRY(side_tail(0));
  } else {
    TRY(side_core(0));
  }
  if (nw > 1) TRY(side_core(1));
  tm.mark();
  HIPCHK(hipStreamWaitEvent(R.st, h->tabs, 0));
  TRY(stage_dft(R, true, false));
  tm.mark();
  const Basis xb{at<char>(R.ws, R.L.zg), 1, (long)R.P.ngg};
  TRY(stage_gram(R, xb));
  tm.mark();
  for (int k = 0; k < nw; ++k) {
    Timer dummy{h, false};
    Timer& t = (k == nw - 1) ? tm : dummy;
    HIPCHK(hipStreamWaitEvent(R.st, h->m_ready[k & 1], 0));
    TRY(stage_core_algebra(R, mbuf[k & 1], h->m_used[k & 1]));
    if (k + 2 < nw) TRY(side_core(k + 2));
    t.mark();
    void* out = reinterpret_cast<char*>(eps_inv) + (size_t)k * ng * ng * 16;
    TRY(stage_out(R, xb, out, t));
    t.mark();
  }
  HIPCHK(hipEventRecord(h->join, side));
  HIPCHK(hipStreamWaitEvent(R.st, h->join, 0));
  return ISDF_OK;
}

// ---- COHSEX self-energy diagonals (Algorithm 3, steps 2 and 4-7) ------------------
// Two more pair sets, each with its own points: vn (occupied x all states) and nn
// (all x all).  For a set s with points r_mu^s:
//   S_s = C_s C_s^H and Z_s = M_s C_s^H (the least-squares fit, as for the vc set),
//   X_s = V^{1/2} F Z_s on the plane-wave list, A_s = X_s^H X (X of the vc set),
//   W_s = -S_s^{-1} A_s H^{-1} A_s^H S_s^{-1}, which is Algorithm 3's
//         (P_s^H V P_vc) K (P_s^H V P_vc)^H with P = Theta = Z S^{-1} and
//         K = (M^{-1} - U^H U)^{-1} = -S H^{-1} S, H = X^H X - S M^{-1} S;
//   V_vn = S_vn^{-1} X_vn^H X_vn S_vn^{-1} (the bare exchange on the vn points);
//   then eq. Hadamard: Sigma(n) = coef diag(Psi_s^H (W_s (.) G_set) Psi_s)(n).
// All N_mu-sized algebra runs in FP64; the contractions over the grid and the
// plane waves in the mode's precision (BF16x3: FP32).
struct SigmaLayout {
  size_t mu_vn = 0, mu_nn = 0, pm = 0, pm32 = 0, s = 0, lin = 0, a = 0, q = 0, b = 0, q2 = 0, w = 0, g = 0,
         e = 0, xt = 0, t2 = 0, zt = 0, total = 0;
  size_t t2_bytes = 0;
};

// the sigma region starts at `base` (the end of the eps~^{-1} layout)
SigmaLayout make_sigma_layout(const Problem& P, int nd, int nvn, int nnn, size_t base) {
  SigmaLayout S;
  size_t off = base;
  auto take = [&](size_t bytes) { size_t o = off; off += up(std::max<size_t>(bytes, 1)); return o; };
  const size_t z = 16, el = P.m32 ? 8 : 16;
  const size_t nm = (size_t)std::max(nvn, nnn);
  S.mu_vn = take((size_t)nvn * 4);
  S.mu_nn = take((size_t)nnn * 4);
  S.pm = take((size_t)P.ns * nm * z);
  if (P.m32) S.pm32 = take((size_t)P.ns * nm * 8);
  S.s = take(nm * nm * z);
  S.lin = take(linalg_scratch_bytes((int)nm));
  S.a = take(nm * P.nmu * z);
  S.q = take(nm * P.nmu * z);
  S.b = take(nm * nm * z);
  S.q2 = take(nm * nm * z);
  S.w = take(nm * nm * z);
  S.g = take(nm * nm * z);
  S.e = take(nm * P.ns * z);
  S.xt = take(nm * P.ng * el);
  S.t2_bytes = std::max(nm * P.n2 * nd, (size_t)std::min(DFT_MAX_ZBLOCKS, P.n2) * nm * P.ng) * el;
  S.t2 = take(S.t2_bytes);
  S.zt = take(nm * P.nr * el);
  S.total = off - base;
  return S;
}

isdf_status check_set_points(isdf_handle h, const Problem& P, const int32_t* mu, int nmu, long pairs, const char* what) {
  if (!mu) return fail(h, ISDF_E_ARG, std::string(what) + " is NULL");
  if (nmu < 1) return fail(h, ISDF_E_ARG, std::string(what) + ": need at least one point");
  if ((long)nmu > pairs || (long)nmu > P.nr)
    return fail(h, ISDF_E_ARG, std::string(what) + ": more points than pair functions or grid points (S would be singular)");
  std::vector<int32_t> v(mu, mu + nmu);
  std::sort(v.begin(), v.end());
  if (v.front() < 0 || v.back() >= P.nr) return fail(h, ISDF_E_ARG, std::string(what) + " out of range");
  for (int i = 1; i < nmu; ++i)
    if (v[i] == v[i - 1]) return fail(h, ISDF_E_ARG, std::string(what) + " has duplicate points");
  return ISDF_OK;
}

// One pair set: na states in the first range (occupied: nv, or all: ns), all states in
// the second; sigma terms written to out_terms[k] for each (coef, use_w) requested.
isdf_status enqueue_sigma_set(Run& R, const SigmaLayout& S, const int* mu, int nmu, int na, bool with_exchange,
                              double* out_sx, double* out_x, double* out_coh) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  const Prec cp = P.prec == P64 ? P64 : P32;
  const int ns = P.ns, n = P.nmu, ng = P.ng;
  const long m2 = (long)nmu * nmu;
  void* pm = at<char>(R.ws, S.pm);
  void* sw = at<char>(R.ws, S.s);
  HIPCHK(gather_points(R.psi, P.nr, ns, mu, nmu, pm, R.st));
  // S_s^T = conj(S_s) on the points, then Sw = -(S_s^T)^{-1} = -conj(S_s^{-1})
  HIPCHK(zpair(P64, nmu, nmu, na, na + ns, pm, nmu, pm, nmu, false, sw, nmu, false, R.st, 1, 0));
  HIPCHK(sweep_inverse(nmu, sw, at<char>(R.ws, S.lin), &R.sb->status, R.st));
  // Z_s^T [mu][r] over the grid, then X_s^T = (V^{1/2} F Z_s)^T [mu][g]
  void* zt = at<char>(R.ws, S.zt);
  if (cp == P64) {
    HIPCHK(zpair(P64, nmu, (int)P.nr, na, na + ns, pm, nmu, R.psi, P.nr, false, zt, P.nr, false, R.st, 1, 0));
  } else {
    void* pm32 = at<char>(R.ws, S.pm32);
    HIPCHK(convert_z(pm, false, pm32, true, (long)ns * nmu, R.st));
    HIPCHK(zpair(P32, nmu, (int)P.nr, na, na + ns, pm32, nmu, R.psi, P.nr, true, zt, P.nr, true, R.st,
                 R.tune.wg_per_cu, 0));
  }
  DftPlan dp = make_plan(R);
  dp.nmu = nmu;
  void* xt = at<char>(R.ws, S.xt);
  TRY(dft_apply(R, dp, zt, at<char>(R.ws, S.t2), S.t2_bytes, xt, at<double>(R.ws, L.sqrtv)));
  // A_s = X_s^H X (N_mu^s x N_mu), over the plane waves
  void* a = at<char>(R.ws, S.a);
  {
    GemmDesc d;
    d.M = nmu; d.N = n; d.K = ng;
    d.A = xt; d.sam = ng; d.sak = 1; d.conjA = true; d.a32 = P.m32;
    d.B = at<char>(R.ws, L.zg); d.sbk = 1; d.sbn = P.ngg; d.b32 = P.m32;
    d.C = a; d.ldc = n;
    HIPCHK(gemm(cp, d, R.st));
  }
  // B_s = A_s H^{-1} A_s^H with H^{-1} = talpha * tmat (FP64)
  void* q = at<char>(R.ws, S.q);
  void* b = at<char>(R.ws, S.b);
  {
    GemmDesc d;
    d.M = nmu; d.N = n; d.K = n;
    d.A = a; d.sam = n; d.sak = 1;
    d.B = R.tmat; d.sbk = n; d.sbn = 1;
    d.C = q; d.ldc = n; d.alpha = R.talpha;
    HIPCHK(gemm(P64, d, R.st));
    GemmDesc e;
    e.M = e.N = nmu; e.K = n;
    e.A = q; e.sam = n; e.sak = 1;
    e.B = a; e.sbk = 1; e.sbn = n; e.conjB = true;
    e.C = b; e.ldc = nmu; e.herm = true;
    HIPCHK(gemm(P64, e, R.st));
  }
  // sandwich: out = alpha S_s^{-1} in S_s^{-1} = alpha conj(Sw) in conj(Sw)
  void* q2 = at<char>(R.ws, S.q2);
  void* w = at<char>(R.ws, S.w);
  auto sandwich = [&](const void* in, double alpha, void* out) -> isdf_status {
    GemmDesc d;
    d.M = d.N = d.K = nmu;
    d.A = in; d.sam = nmu; d.sak = 1;
    d.B = sw; d.sbk = nmu; d.sbn = 1; d.conjB = true;
    d.C = q2; d.ldc = nmu;
    HIPCHK(gemm(P64, d, R.st));
    GemmDesc e;
    e.M = e.N = e.K = nmu;
    e.A = sw; e.sam = nmu; e.sak = 1; e.conjA = true;
    e.B = q2; e.sbk = nmu; e.sbn = 1;
    e.C = out; e.ldc = nmu; e.alpha = alpha; e.herm = true;
    HIPCHK(gemm(P64, e, R.st));
    return ISDF_OK;
  };
  // G_set(mu, nu) = sum_{i < na} psi_i(r_mu) conj(psi_i(r_nu))
  void* g = at<char>(R.ws, S.g);
  {
    GemmDesc d;
    d.M = d.N = nmu; d.K = na;
    d.A = pm; d.sam = 1; d.sak = nmu;
    d.B = pm; d.sbk = nmu; d.sbn = 1; d.conjB = true;
    d.C = g; d.ldc = nmu; d.herm = true;
    HIPCHK(gemm(P64, d, R.st));
  }
  // Sigma(n) = coef Re diag(Psi^H (Y (.) G) Psi), Y = W_s or V_vn
  void* ebuf = at<char>(R.ws, S.e);
  auto diag_term = [&](const void* y, double coef, double* out) -> isdf_status {
    HIPCHK(mul_z(y, g, q2, m2, R.st));
    GemmDesc d;   // E = (Y (.) G) Psi, Psi(nu, n) = pm[n][nu]
    d.M = nmu; d.N = ns; d.K = nmu;
    d.A = q2; d.sam = nmu; d.sak = 1;
    d.B = pm; d.sbk = 1; d.sbn = nmu;
    d.C = ebuf; d.ldc = ns;
    HIPCHK(gemm(P64, d, R.st));
    HIPCHK(sigma_diag(pm, ebuf, nmu, ns, coef, out, R.st));
    return ISDF_OK;
  };
  TRY(sandwich(b, -1.0, w));                       // W_s
  if (with_exchange) {
    TRY(diag_term(w, -1.0, out_sx));               // Sigma_SEX_X = -diag(Psi^H (W_vn (.) G_v) Psi)
    GemmDesc d;                                    // X_vn^H X_vn (Hermitian, over the plane waves)
    d.M = d.N = nmu; d.K = ng;
    d.A = xt; d.sam = ng; d.sak = 1; d.conjA = true; d.a32 = P.m32;
    d.B = xt; d.sbk = 1; d.sbn = ng; d.b32 = P.m32;
    d.C = b; d.ldc = nmu; d.herm = true;
    HIPCHK(gemm(cp, d, R.st));
    TRY(sandwich(b, 1.0, w));                      // V_vn
    TRY(diag_term(w, -1.0, out_x));                // Sigma_X
  } else {
    TRY(diag_term(w, 0.5, out_coh));               // Sigma_COH = 1/2 diag(Psi^H (W_nn (.) G_all) Psi)
  }
  return ISDF_OK;
}

}  // namespace


// ---- the workspace of the allocation-free entry point ----------------------------
// One array per GPU, a file-scope device variable: the runtime places a copy on each
// device the library runs on and keeps it until the process ends.  In host code its
// name is only a stand-in; the device address is taken once per device, with that
// device current, by scratch_setup (from isdf_create), and only that address is used.
static __device__ __align__(256) unsigned char scratch[ISDF_SCRATCH_MAX_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_addr[SCRATCH_MAX_DEVICES] = {};

// the calling thread's current device must be `device`
hipError_t scratch_setup(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (scratch_addr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr || (reinterpret_cast<uintptr_t>(ptr) & (ALIGN - 1)) != 0) return hipErrorInvalidSymbol;
  scratch_addr[device] = ptr;
  return hipSuccess;
}

void* scratch_of(int device) {
  if (device < 0 || device >= SCRATCH_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  return scratch_addr[device];
}
}  // namespace

extern "C" {

const char* isdf_version(void) { return "isdf-smw-gfx950 0.1"; }

isdf_status isdf_create(isdf_handle* out, int device, void* stream) {
  if (!out) return ISDF_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return ISDF_E_ARG;
  isdf_handle h = new isdf_handle_s;
  h->device = device;
  h->stream = (hipStream_t)stream;
  if (hipSetDevice(device) != hipSuccess) { delete h; return ISDF_E_DEVICE; }
  if (scratch_setup(device) != hipSuccess) { delete h; return ISDF_E_DEVICE; }
  for (auto& e : h->ev)
    if (hipEventCreate(&e) != hipSuccess) { delete h; return ISDF_E_DEVICE; }
  for (hipEvent_t* e : {&h->fork, &h->join, &h->core0, &h->zdone, &h->zops, &h->tabs, &h->mfork, &h->mdone, &h->m_ready[0],
                        &h->m_ready[1], &h->m_used[0], &h->m_used[1]})
    if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) { delete h; return ISDF_E_DEVICE; }
  // default priority, non-blocking with respect to the legacy default stream
  if (hipStreamCreateWithFlags(&h->side, hipStreamNonBlocking) != hipSuccess) { delete h; return ISDF_E_DEVICE; }
  h->pinned_bytes = 1 << 20;
  if (hipHostMalloc(&h->pinned, h->pinned_bytes, hipHostMallocDefault) != hipSuccess) {
    (void)isdf_destroy(h);
    return ISDF_E_DEVICE;
  }
  *out = h;
  return ISDF_OK;
}

isdf_status isdf_destroy(isdf_handle h) {
  if (!h) return ISDF_OK;
  (void)hipStreamSynchronize(h->stream);
  if (h->side) {
    (void)hipStreamSynchronize(h->side);
    (void)hipStreamDestroy(h->side);
  }
  for (auto& e : h->ev) if (e) (void)hipEventDestroy(e);
  for (hipEvent_t e : {h->fork, h->join, h->core0, h->zdone, h->zops, h->tabs, h->mfork, h->mdone, h->m_ready[0], h->m_ready[1],
                       h->m_used[0], h->m_used[1]})
    if (e) (void)hipEventDestroy(e);
  if (h->pinned) (void)hipHostFree(h->pinned);
  delete h;
  return ISDF_OK;
}

isdf_status isdf_set_stream(isdf_handle h, void* stream) {
  if (!h) return ISDF_E_ARG;
  h->stream = (hipStream_t)stream;
  return ISDF_OK;
}

const char* isdf_last_error(isdf_handle h) { return h ? h->err.c_str() : "null handle"; }

isdf_status isdf_workspace_bytes(const isdf_problem* prob, int32_t n_mu, int32_t ng, int32_t n_omega,
                                 size_t* bytes) {
  if (!bytes) return ISDF_E_ARG;
  Problem P;
  isdf_status s = check_problem(nullptr, prob, P);
  if (s != ISDF_OK) return s;
  if (n_mu < 1 || ng < 1 || n_omega < 0) return ISDF_E_ARG;
  P.nmu = n_mu;
  P.ng = ng;
  P.nomega = n_omega;
  P.ngg = P.full_gram ? (int)P.nr : ng;
  // worst-case DFT bookkeeping for ngg vectors: every list at most min(ngg, n_d), pairs at most ngg
  const int kx = std::min(P.ngg, P.n0), ky = std::min(P.ngg, P.n1), kz = std::min(P.ngg, P.n2);
  const int nd = (int)std::min<long>(P.ngg, (long)P.n0 * P.n1);
  *bytes = make_layout(P, kx, ky, kz, nd).total;
  return ISDF_OK;
}

isdf_status isdf_check_inputs(const isdf_problem* prob, const double* energies, const int32_t* mu_idx,
                              int32_t n_mu, const int32_t* miller, int32_t ng, const double* omega,
                              int32_t n_omega, char* msg, size_t msg_len) {
  isdf_handle_s tmp;
  isdf_handle h = &tmp;
  auto ret = [&](isdf_status s) {
    if (msg && msg_len) {
      std::strncpy(msg, tmp.err.c_str(), msg_len - 1);
      msg[msg_len - 1] = 0;
    }
    return s;
  };
  Problem P;
  isdf_status s = begin(h, prob, P, n_mu, ng, n_omega);
  if (s != ISDF_OK) return ret(s);
  if (n_omega < 0 || (n_omega > 0 && !omega)) return ret(fail(h, ISDF_E_ARG, "omega list invalid"));
  for (int k = 0; k < n_omega; ++k)
    if (!(omega[k] >= 0.0) || !std::isfinite(omega[k])) return ret(fail(h, ISDF_E_ARG, "omega must be finite and >= 0"));
  if ((s = check_points(h, P, mu_idx, n_mu)) != ISDF_OK) return ret(s);
  if ((s = check_miller(h, P, miller, ng)) != ISDF_OK) return ret(s);
  if ((s = check_energies(h, P, energies)) != ISDF_OK) return ret(s);
  return ret(ISDF_OK);
}

isdf_status isdf_gvectors(const isdf_problem* prob, int32_t ng, int32_t* miller_out) {
  Problem P;
  isdf_status s = check_problem(nullptr, prob, P);
  if (s != ISDF_OK) return s;
  if (!miller_out || ng < 1 || (long)ng > P.nr) return ISDF_E_ARG;
  struct M { long m2; int x, y, z; };
  std::vector<M> all;
  all.reserve(P.nr);
  for (int x = -(P.n0 / 2); x < P.n0 - P.n0 / 2; ++x)
    for (int y = -(P.n1 / 2); y < P.n1 - P.n1 / 2; ++y)
      for (int z = -(P.n2 / 2); z < P.n2 - P.n2 / 2; ++z)
        all.push_back({(long)x * x + (long)y * y + (long)z * z, x, y, z});
  std::partial_sort(all.begin(), all.begin() + ng, all.end(), [](const M& a, const M& b) {
    if (a.m2 != b.m2) return a.m2 < b.m2;
    if (a.x != b.x) return a.x < b.x;
    if (a.y != b.y) return a.y < b.y;
    return a.z < b.z;
  });
  for (int g = 0; g < ng; ++g) {
    miller_out[3 * g] = all[g].x;
    miller_out[3 * g + 1] = all[g].y;
    miller_out[3 * g + 2] = all[g].z;
  }
  return ISDF_OK;
}

isdf_status isdf_eps_inv(isdf_handle h, const isdf_problem* prob, const void* psi, const double* energies,
                         const int32_t* mu_idx, int32_t n_mu, const int32_t* miller, int32_t ng,
                         const double* omega, int32_t n_omega, void* workspace, size_t ws_bytes,
                         void* eps_inv, isdf_report* rep) {
  if (!h) return ISDF_E_ARG;
  if (n_omega < 0 || (n_omega > 0 && !omega)) return fail(h, ISDF_E_ARG, "omega list invalid");
  for (int k = 0; k < n_omega; ++k)
    if (!(omega[k] >= 0.0) || !std::isfinite(omega[k])) return fail(h, ISDF_E_ARG, "omega must be finite and >= 0");
  if (!eps_inv) return fail(h, ISDF_E_ARG, "eps_inv is NULL");
  if (!energies) return fail(h, ISDF_E_ARG, "energies is NULL");
  if (!miller) return fail(h, ISDF_E_ARG, "miller is NULL");
  Run R;
  Uploader upl;
  DftIndex ix;
  std::vector<int> idxbuf;
  TRY(setup_common(R, h, prob, psi, mu_idx, n_mu, miller, ng, energies, n_omega, workspace, ws_bytes, upl, ix, idxbuf));
  if (R.P.core_method == 1 && n_omega > 0)
    return fail(h, ISDF_E_UNSUPPORTED, "the contour-integral core is static (n_omega = 0)");
  HIPCHK(hipSetDevice(h->device));
  TRY(upl.run());
  TRY(clear_status(R));
  Timer tm{h, rep && rep->want_timing != 0};
  tm.mark();
  TRY(enqueue_eps_inv(R, psi, omega, n_omega, eps_inv, tm));
  return finish(R, rep, tm);
}

isdf_status isdf_eps_inv_noalloc(isdf_handle h, const isdf_problem* prob, const void* psi, const double* energies,
                                 const int32_t* mu_idx, int32_t n_mu, const int32_t* miller, int32_t ng,
                                 const double* omega, int32_t n_omega, void* eps_inv, isdf_report* rep) {
  if (!h) return ISDF_E_ARG;
  if (n_omega < 0 || (n_omega > 0 && !omega)) return fail(h, ISDF_E_ARG, "omega list invalid");
  for (int k = 0; k < n_omega; ++k)
    if (!(omega[k] >= 0.0) || !std::isfinite(omega[k])) return fail(h, ISDF_E_ARG, "omega must be finite and >= 0");
  if (!eps_inv) return fail(h, ISDF_E_ARG, "eps_inv is NULL");
  if (!energies) return fail(h, ISDF_E_ARG, "energies is NULL");
  if (!miller) return fail(h, ISDF_E_ARG, "miller is NULL");
  void* ws = scratch_of(h->device);
  if (!ws) return fail(h, ISDF_E_DEVICE, "the device's scratch array was not set up by isdf_create");
  Run R;
  Uploader upl;
  upl.no_alloc = true;
  DftIndex ix;
  std::vector<int> idxbuf;
  const isdf_status s0 = setup_common(R, h, prob, psi, mu_idx, n_mu, miller, ng, energies, n_omega, ws,
                                      ISDF_SCRATCH_MAX_BYTES, upl, ix, idxbuf);
  if (s0 == ISDF_E_WORKSPACE)
    return fail(h, ISDF_E_WORKSPACE, "the problem needs " + std::to_string(R.L.total) +
                " bytes of workspace; the allocation-free entry point holds at most " +
                std::to_string((size_t)ISDF_SCRATCH_MAX_BYTES) + " (use isdf_eps_inv with a caller workspace)");
  TRY(s0);
  if (R.P.core_method == 1 && n_omega > 0)
    return fail(h, ISDF_E_UNSUPPORTED, "the contour-integral core is static (n_omega = 0)");
  HIPCHK(hipSetDevice(h->device));
  TRY(upl.run());
  TRY(clear_status(R));
  Timer tm{h, rep && rep->want_timing != 0};
  tm.mark();
  TRY(enqueue_eps_inv(R, psi, omega, n_omega, eps_inv, tm));
  return finish(R, rep, tm);
}

isdf_status isdf_sigma_workspace_bytes(const isdf_problem* prob, int32_t n_mu, int32_t ng, int32_t n_mu_vn,
                                       int32_t n_mu_nn, size_t* bytes) {
  if (!bytes || n_mu_vn < 1 || n_mu_nn < 1) return ISDF_E_ARG;
  size_t main = 0;
  TRY(isdf_workspace_bytes(prob, n_mu, ng, 0, &main));
  Problem P;
  TRY(check_problem(nullptr, prob, P));
  P.nmu = n_mu;
  P.ng = P.ngg = ng;
  const int nd = (int)std::min<long>(ng, (long)P.n0 * P.n1);
  *bytes = main + make_sigma_layout(P, nd, n_mu_vn, n_mu_nn, main).total;
  return ISDF_OK;
}

isdf_status isdf_sigma_cohsex(isdf_handle h, const isdf_problem* prob, const void* psi, const double* energies,
                              const int32_t* mu_idx, int32_t n_mu, const int32_t* mu_vn, int32_t n_mu_vn,
                              const int32_t* mu_nn, int32_t n_mu_nn, const int32_t* miller, int32_t ng,
                              void* workspace, size_t ws_bytes, void* eps_inv, double* sigma, isdf_report* rep) {
  if (!h) return ISDF_E_ARG;
  if (!eps_inv) return fail(h, ISDF_E_ARG, "eps_inv is NULL");
  if (!sigma) return fail(h, ISDF_E_ARG, "sigma is NULL");
  if (!energies) return fail(h, ISDF_E_ARG, "energies is NULL");
  if (!miller) return fail(h, ISDF_E_ARG, "miller is NULL");
  if (prob && prob->coulomb_sum != 0)
    return fail(h, ISDF_E_UNSUPPORTED, "the self-energies use the plane-wave list's Coulomb operator (coulomb_sum = 0)");
  Run R;
  Uploader upl;
  DftIndex ix;
  std::vector<int> idxbuf;
  // the eps~^{-1} layout first, checked against the whole workspace below
  TRY(setup_common(R, h, prob, psi, mu_idx, n_mu, miller, ng, energies, 0, workspace, ws_bytes, upl, ix, idxbuf));
  const Problem& P = R.P;
  TRY(check_set_points(h, P, mu_vn, n_mu_vn, (long)P.nv * P.ns, "mu_vn"));
  TRY(check_set_points(h, P, mu_nn, n_mu_nn, (long)P.ns * P.ns, "mu_nn"));
  const SigmaLayout S = make_sigma_layout(P, R.L.nd, n_mu_vn, n_mu_nn, R.L.total);
  TRY(check_ws(h, workspace, ws_bytes, R.L.total + S.total));
  upl.add(S.mu_vn, mu_vn, (size_t)n_mu_vn * 4);
  upl.add(S.mu_nn, mu_nn, (size_t)n_mu_nn * 4);
  HIPCHK(hipSetDevice(h->device));
  TRY(upl.run());
  TRY(clear_status(R));
  Timer tm{h, rep && rep->want_timing != 0};
  tm.mark();
  TRY(enqueue_eps_inv(R, psi, nullptr, 0, eps_inv, tm));
  const int ns = P.ns;
  TRY(enqueue_sigma_set(R, S, at<int>(workspace, S.mu_vn), n_mu_vn, P.nv, true, sigma, sigma + ns, nullptr));
  TRY(enqueue_sigma_set(R, S, at<int>(workspace, S.mu_nn), n_mu_nn, ns, false, nullptr, nullptr, sigma + 2 * ns));
  return finish(R, rep, tm);
}

isdf_status isdf_fit_theta(isdf_handle h, const isdf_problem* prob, const void* psi, const int32_t* mu_idx,
                           int32_t n_mu, void* workspace, size_t ws_bytes, void* theta) {
  if (!h) return ISDF_E_ARG;
  if (!theta) return fail(h, ISDF_E_ARG, "theta is NULL");
  Run R;
  Uploader upl;
  DftIndex ix;
  std::vector<int> idxbuf;
  TRY(setup_common(R, h, prob, psi, mu_idx, n_mu, nullptr, 1, nullptr, 0, workspace, ws_bytes, upl, ix, idxbuf));
  HIPCHK(hipSetDevice(h->device));
  TRY(upl.run());
  TRY(clear_status(R));
  TRY(prepare_psi(R, psi));
  TRY(stage_points(R));
  TRY(stage_s(R, R.st, R.L.lin, true));
  TRY(stage_z_operands(R));
  TRY(stage_z(R));
  const Problem& P = R.P;
  // Theta^T(nu, r) = sum_mu S^{-1}(mu, nu) Zt(mu, r), S^{-1}(mu, nu) = -Sw[nu][mu]
  GemmDesc d;
  d.M = P.nmu; d.N = (int)P.nr; d.K = P.nmu;
  d.A = at<char>(workspace, R.L.s); d.sam = P.nmu; d.sak = 1;
  d.B = at<char>(workspace, R.L.zt); d.sbk = P.nr; d.sbn = 1; d.b32 = P.m32;
  d.C = theta; d.ldc = P.nr; d.alpha = -1.0;
  HIPCHK(gemm(P.prec == P64 ? P64 : P32, d, R.st));
  Timer tm{h, false};
  return finish(R, nullptr, tm);
}

isdf_status isdf_core_m(isdf_handle h, const isdf_problem* prob, const void* psi, const double* energies,
                        const int32_t* mu_idx, int32_t n_mu, double omega, void* workspace,
                        size_t ws_bytes, void* m_out) {
  if (!h) return ISDF_E_ARG;
  if (!m_out) return fail(h, ISDF_E_ARG, "m_out is NULL");
  if (!energies) return fail(h, ISDF_E_ARG, "energies is NULL");
  if (!(omega >= 0.0) || !std::isfinite(omega)) return fail(h, ISDF_E_ARG, "omega must be finite and >= 0");
  Run R;
  Uploader upl;
  DftIndex ix;
  std::vector<int> idxbuf;
  TRY(setup_common(R, h, prob, psi, mu_idx, n_mu, nullptr, 1, energies, 0, workspace, ws_bytes, upl, ix, idxbuf));
  HIPCHK(hipSetDevice(h->device));
  TRY(upl.run());
  TRY(clear_status(R));
  TRY(prepare_psi(R, psi));
  HIPCHK(gather_points(R.psi, R.P.nr, R.P.ns, R.mu, R.P.nmu, at<char>(workspace, R.L.pm), R.st));
  TRY(stage_core(R, omega, m_out, nullptr, R.st));
  Timer tm{h, false};
  return finish(R, nullptr, tm);
}

isdf_status isdf_coulomb_u(isdf_handle h, const isdf_problem* prob, const void* psi, const int32_t* mu_idx,
                           int32_t n_mu, const int32_t* miller, int32_t ng, void* workspace,
                           size_t ws_bytes, void* u_out) {
  if (!h) return ISDF_E_ARG;
  if (!u_out) return fail(h, ISDF_E_ARG, "u_out is NULL");
  if (!miller) return fail(h, ISDF_E_ARG, "miller is NULL");
  Run R;
  Uploader upl;
  DftIndex ix;
  std::vector<int> idxbuf;
  TRY(setup_common(R, h, prob, psi, mu_idx, n_mu, miller, ng, nullptr, 0, workspace, ws_bytes, upl, ix, idxbuf));
  HIPCHK(hipSetDevice(h->device));
  TRY(upl.run());
  TRY(clear_status(R));
  TRY(prepare_psi(R, psi));
  TRY(stage_points(R));
  TRY(stage_s(R, R.st, R.L.lin, true));
  TRY(stage_z_operands(R));
  TRY(stage_z(R));
  TRY(stage_dft(R, true));
  TRY(stage_u(R));
  HIPCHK(convert_z(at<char>(workspace, R.L.u), R.P.m32, u_out, false, (long)ng * n_mu, R.st));
  Timer tm{h, false};
  return finish(R, nullptr, tm);
}

isdf_status isdf_smw_apply(isdf_handle h, const isdf_problem* prob, const void* u, const void* m,
                           int32_t n_mu, int32_t ng, void* workspace, size_t ws_bytes, void* eps_inv,
                           isdf_report* rep) {
  if (!h) return ISDF_E_ARG;
  if (!u || !m || !eps_inv) return fail(h, ISDF_E_ARG, "u, m and eps_inv must be non-NULL");
  Run R;
  TRY(begin(h, prob, R.P, n_mu, ng, 0));
  if (n_mu < 1 || ng < 1) return fail(h, ISDF_E_ARG, "n_mu and ng must be >= 1");
  R.L = make_layout(R.P, 1, 1, 1, 1);
  TRY(check_ws(h, workspace, ws_bytes, R.L.total));
  R.h = h; R.ws = workspace; R.st = h->stream;
  R.sb = at<StatusBlock>(workspace, R.L.status);
  HIPCHK(hipSetDevice(h->device));
  TRY(clear_status(R));
  Timer tm{h, rep && rep->want_timing != 0};
  tm.mark();
  HIPCHK(convert_z(u, false, at<char>(workspace, R.L.u), R.P.m32, (long)ng * n_mu, R.st));
  HIPCHK(scale_z(m, at<char>(workspace, R.L.l), (long)n_mu * n_mu, -1.0, R.st));  // -M
  HIPCHK(sweep_inverse(n_mu, at<char>(workspace, R.L.l), at<char>(workspace, R.L.lin), &R.sb->status, R.st));
  tm.mark();
  tm.mark();
  const Basis ub{at<char>(workspace, R.L.u), (long)n_mu, 1};
  TRY(stage_gram(R, ub));
  tm.mark();
  TRY(stage_core_algebra(R, at<char>(workspace, R.L.l), nullptr));
  tm.mark();
  TRY(stage_out(R, ub, eps_inv, tm));
  tm.mark();
  return finish(R, rep, tm);
}

// ---- plans: validated, uploaded once; enqueue-only execution -------------------------------
struct isdf_plan_s {
  isdf_handle h = nullptr;
  Problem P;
  Layout L;
  Tune tune;
  int n_omega = 0;
  void* dev = nullptr;  // caller's table buffer: status block, point indices, Miller list, reciprocal basis, DFT tables
  size_t off_mu = 0, off_miller = 0, off_recip = 0, off_idx = 0;
  // per-call stage timing (isdf_plan_time_stages): 10 events per call since the last sync
  bool timing = false;
  std::vector<hipEvent_t> tev;
  int tn = 0, tmarks = 0;
  hipStream_t last = nullptr;   // stream of the last enqueued call (isdf_plan_sync waits for it)
  bool last_set = false;
};

namespace {

// Host image of a plan's device tables (validated problem, points, plane waves).
struct PlanTables {
  Problem P;
  Layout L;
  size_t off_mu = 0, off_miller = 0, off_recip = 0, off_idx = 0, total = 0;
  std::vector<char> host;
};

isdf_status plan_tables(isdf_handle h, const isdf_problem* prob, const int32_t* mu_idx, int32_t n_mu,
                        const int32_t* miller, int32_t ng, int32_t n_omega, PlanTables& T) {
  if (n_omega < 0) return fail(h, ISDF_E_ARG, "n_omega must be >= 0");
  Problem& P = T.P;
  TRY(begin(h, prob, P, n_mu, ng, n_omega));
  if (P.core_method == 1)
    return fail(h, ISDF_E_UNSUPPORTED, "plans take device energies; the contour-integral core needs them on the host");
  TRY(check_points(h, P, mu_idx, n_mu));
  TRY(check_miller(h, P, miller, ng));
  std::vector<int32_t> full;
  if (P.full_gram) {
    full = full_grid_list(miller, ng, P.n0, P.n1, P.n2);
    miller = full.data();
  }
  DftIndex ix = dft_index(miller, P.ngg);
  if (!dft_supported(P.n0, P.n1, P.n2, (int)ix.xl.size(), (int)ix.yl.size(), P.prec == P64 ? P64 : P32))
    return fail(h, ISDF_E_UNSUPPORTED, "grid axis above 64 points: the DFT keeps an x-y slab in LDS and a z-line per wave");
  std::vector<int> idxbuf;
  for (auto* v : {&ix.xl, &ix.yl, &ix.zl, &ix.d_ax, &ix.d_by, &ix.g_d, &ix.g_cz, &ix.dmap, &ix.gd_off, &ix.gd_list})
    idxbuf.insert(idxbuf.end(), v->begin(), v->end());
  T.L = make_layout(P, (int)ix.xl.size(), (int)ix.yl.size(), (int)ix.zl.size(), (int)ix.d_ax.size());
  size_t off = up(sizeof(StatusBlock));
  T.off_mu = off; off += up((size_t)n_mu * 4);
  T.off_miller = off; off += up((size_t)P.ngg * 12);
  T.off_recip = off; off += up(9 * 8);
  T.off_idx = off; off += up(idxbuf.size() * 4);
  T.total = off;
  T.host.assign(off, 0);
  std::memcpy(T.host.data() + T.off_mu, mu_idx, (size_t)n_mu * 4);
  std::memcpy(T.host.data() + T.off_miller, miller, (size_t)P.ngg * 12);
  std::memcpy(T.host.data() + T.off_recip, P.recip, 9 * 8);
  std::memcpy(T.host.data() + T.off_idx, idxbuf.data(), idxbuf.size() * 4);
  return ISDF_OK;
}

}  // namespace

isdf_status isdf_plan_table_bytes(const isdf_problem* prob, const int32_t* mu_idx, int32_t n_mu,
                                  const int32_t* miller, int32_t ng, int32_t n_omega, size_t* bytes) {
  if (!bytes) return ISDF_E_ARG;
  isdf_handle_s tmp;
  PlanTables T;
  TRY(plan_tables(&tmp, prob, mu_idx, n_mu, miller, ng, n_omega, T));
  *bytes = T.total;
  return ISDF_OK;
}

isdf_status isdf_plan_create(isdf_handle h, const isdf_problem* prob, const int32_t* mu_idx, int32_t n_mu,
                             const int32_t* miller, int32_t ng, int32_t n_omega, void* tables,
                             size_t table_bytes, isdf_plan* out) {
  if (!h || !out) return ISDF_E_ARG;
  *out = nullptr;
  PlanTables T;
  TRY(plan_tables(h, prob, mu_idx, n_mu, miller, ng, n_omega, T));
  if (!tables) return fail(h, ISDF_E_WORKSPACE, "plan table buffer is NULL");
  if (reinterpret_cast<uintptr_t>(tables) % ALIGN) return fail(h, ISDF_E_WORKSPACE, "plan table buffer not 256-byte aligned");
  if (table_bytes < T.total)
    return fail(h, ISDF_E_WORKSPACE, "plan table buffer too small: need " + std::to_string(T.total) + " bytes");
  HIPCHK(hipSetDevice(h->device));
  HIPCHK(hipMemcpyAsync(tables, T.host.data(), T.total, hipMemcpyHostToDevice, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  isdf_plan pl = new isdf_plan_s;
  pl->h = h;
  pl->P = T.P;
  pl->L = T.L;
  pl->n_omega = n_omega;
  pl->dev = tables;
  pl->off_mu = T.off_mu;
  pl->off_miller = T.off_miller;
  pl->off_recip = T.off_recip;
  pl->off_idx = T.off_idx;
  *out = pl;
  h->err.clear();
  return ISDF_OK;
}

isdf_status isdf_plan_destroy(isdf_plan pl) {
  if (!pl) return ISDF_OK;
  (void)hipSetDevice(pl->h->device);
  (void)hipStreamSynchronize(pl->h->stream);
  if (pl->last_set && pl->last != pl->h->stream) (void)hipStreamSynchronize(pl->last);
  for (hipEvent_t e : pl->tev) (void)hipEventDestroy(e);
  delete pl;
  return ISDF_OK;
}

isdf_status isdf_plan_time_stages(isdf_plan pl, int32_t on) {
  if (!pl || (on != 0 && on != 1)) return ISDF_E_ARG;
  pl->timing = on == 1;
  pl->tn = 0;
  return ISDF_OK;
}

isdf_status isdf_plan_workspace_bytes(isdf_plan pl, size_t* bytes) {
  if (!pl || !bytes) return ISDF_E_ARG;
  *bytes = pl->L.total;
  return ISDF_OK;
}

}  // extern "C"

namespace {

isdf_status plan_check(isdf_plan pl, const void* psi, const double* energies, const double* omega, void* workspace,
                       size_t ws_bytes, void* eps_inv) {
  if (!pl) return ISDF_E_ARG;
  isdf_handle h = pl->h;
  if (!psi) return fail(h, ISDF_E_ARG, "psi is NULL");
  if (!energies) return fail(h, ISDF_E_ARG, "energies is NULL");
  if (!eps_inv) return fail(h, ISDF_E_ARG, "eps_inv is NULL");
  if (pl->n_omega > 0 && !omega) return fail(h, ISDF_E_ARG, "omega list invalid");
  for (int k = 0; k < pl->n_omega; ++k)
    if (!(omega[k] >= 0.0) || !std::isfinite(omega[k])) return fail(h, ISDF_E_ARG, "omega must be finite and >= 0");
  return check_ws(h, workspace, ws_bytes, pl->L.total);
}

isdf_status plan_enqueue(isdf_plan pl, const void* psi, const double* energies, const double* omega,
                         void* workspace, void* eps_inv, bool allow_timing = true) {
  isdf_handle h = pl->h;
  Run R;
  R.h = h;
  R.P = pl->P;
  R.L = pl->L;
  R.ws = workspace;
  R.st = h->stream;
  char* d = reinterpret_cast<char*>(pl->dev);
  R.sb = reinterpret_cast<StatusBlock*>(d);
  R.mu = reinterpret_cast<const int*>(d + pl->off_mu);
  R.e = energies;
  R.miller = reinterpret_cast<const int*>(d + pl->off_miller);
  R.recip = reinterpret_cast<const double*>(d + pl->off_recip);
  R.idx = reinterpret_cast<const int*>(d + pl->off_idx);
  R.tune = pl->tune;
  HIPCHK(hipSetDevice(h->device));
  pl->last = R.st;
  pl->last_set = true;
  if (allow_timing && pl->timing && pl->tn < PLAN_TIMED_CALLS) {
    while ((int)pl->tev.size() < 10 * (pl->tn + 1)) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      pl->tev.push_back(e);
    }
    Timer t{h, true, 0, pl->tev.data() + 10 * pl->tn};
    t.mark();
    R.gap_side = true;
    TRY(enqueue_eps_inv(R, psi, omega, pl->n_omega, eps_inv, t));
    pl->tmarks = t.k;
    ++pl->tn;
    return ISDF_OK;
  }
  R.gap_side = true;
  Timer none{h, false};
  return enqueue_eps_inv(R, psi, omega, pl->n_omega, eps_inv, none);
}

}  // namespace

extern "C" {

isdf_status isdf_plan_eps_inv(isdf_plan pl, const void* psi, const double* energies, const double* omega,
                              void* workspace, size_t ws_bytes, void* eps_inv) {
  TRY(plan_check(pl, psi, energies, omega, workspace, ws_bytes, eps_inv));
  return plan_enqueue(pl, psi, energies, omega, workspace, eps_inv);
}

isdf_status isdf_plan_eps_inv_multi(int32_t count, const isdf_plan* plans, const void* const* psi,
                                    const double* const* energies, const double* const* omega,
                                    void* const* workspace, const size_t* ws_bytes, void* const* eps_inv) {
  if (count < 1 || !plans || !psi || !energies || !workspace || !ws_bytes || !eps_inv) return ISDF_E_ARG;
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return ISDF_E_ARG;
    if (plans[i]->h->device != plans[0]->h->device) return fail(plans[0]->h, ISDF_E_ARG, "plans on different devices");
    TRY(plan_check(plans[i], psi[i], energies[i], omega ? omega[i] : nullptr, workspace[i], ws_bytes[i], eps_inv[i]));
  }
  isdf_handle h0 = plans[0]->h;
  hipStream_t main = h0->stream;
  HIPCHK_H(h0, hipSetDevice(h0->device));
  // Eagerly, every other stream is forked off the first plan's stream, each system
  // is enqueued on its own handle's streams, and they are joined back.  Under a
  // stream capture such a fork would make the handles' second streams join the
  // capture through streams that themselves joined it (a nested fork); that form
  // is refused here.  Systems that should run concurrently inside one graph go
  // through isdf_multi_graph_create instead, which captures each system on its
  // own and copies the captured kernels into one graph.
  bool forks = false;
  for (int i = 0; i < count; ++i) forks = forks || plans[i]->h->stream != main;
  if (forks) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIPCHK_H(h0, hipStreamIsCapturing(main, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return fail(h0, ISDF_E_UNSUPPORTED,
                  "isdf_plan_eps_inv_multi under stream capture needs every plan on the capturing stream "
                  "(use isdf_multi_graph_create for systems that run concurrently in one graph)");
  }
  HIPCHK_H(h0, hipEventRecord(h0->mfork, main));
  for (int i = 0; i < count; ++i) {
    isdf_handle hi = plans[i]->h;
    if (hi->stream != main) HIPCHK_H(hi, hipStreamWaitEvent(hi->stream, h0->mfork, 0));
    TRY(plan_enqueue(plans[i], psi[i], energies[i], omega ? omega[i] : nullptr, workspace[i], eps_inv[i]));
    if (hi->stream != main) {
      HIPCHK_H(hi, hipEventRecord(hi->mdone, hi->stream));
      HIPCHK_H(h0, hipStreamWaitEvent(main, hi->mdone, 0));
    }
  }
  return ISDF_OK;
}

// ---- several systems as one graph ---------------------------------------------------------
// Copies the nodes and edges of `child` into `parent` (no edges to the parent's other
// nodes).  A child graph node runs its graph as one unit, and the HIP runtime runs the
// child graph nodes of one launch one after another, while independent kernel nodes of
// one graph run concurrently: so the captured systems are merged node by node.  Only
// kernel and empty nodes are copied (what a plan call records).  Returns MERGE_OTHER,
// with nothing added, if the graph holds anything else.
enum MergeResult { MERGE_OK, MERGE_OTHER, MERGE_ERROR };
static MergeResult merge_graph(hipGraph_t parent, hipGraph_t child) {
  size_t n = 0;
  if (hipGraphGetNodes(child, nullptr, &n) != hipSuccess) return MERGE_ERROR;
  std::vector<hipGraphNode_t> nodes(n), copies(n);
  if (n && hipGraphGetNodes(child, nodes.data(), &n) != hipSuccess) return MERGE_ERROR;
  std::vector<hipKernelNodeParams> kp(n);
  std::vector<char> is_kernel(n, 0);
  for (size_t i = 0; i < n; ++i) {
    hipGraphNodeType t;
    if (hipGraphNodeGetType(nodes[i], &t) != hipSuccess) return MERGE_ERROR;
    if (t == hipGraphNodeTypeKernel) {
      if (hipGraphKernelNodeGetParams(nodes[i], &kp[i]) != hipSuccess) return MERGE_ERROR;
      is_kernel[i] = 1;
    } else if (t != hipGraphNodeTypeEmpty) {
      return MERGE_OTHER;
    }
  }
  size_t ne = 0;
  if (hipGraphGetEdges(child, nullptr, nullptr, &ne) != hipSuccess) return MERGE_ERROR;
  std::vector<hipGraphNode_t> from(ne), to(ne);
  if (ne && hipGraphGetEdges(child, from.data(), to.data(), &ne) != hipSuccess) return MERGE_ERROR;
  for (size_t i = 0; i < n; ++i) {
    const hipError_t e = is_kernel[i] ? hipGraphAddKernelNode(&copies[i], parent, nullptr, 0, &kp[i])
                                      : hipGraphAddEmptyNode(&copies[i], parent, nullptr, 0);
    if (e != hipSuccess) return MERGE_ERROR;
  }
  std::map<hipGraphNode_t, hipGraphNode_t> map;
  for (size_t i = 0; i < n; ++i) map[nodes[i]] = copies[i];
  for (size_t i = 0; i < ne; ++i) {
    const auto fa = map.find(from[i]), fb = map.find(to[i]);
    if (fa == map.end() || fb == map.end()) return MERGE_ERROR;
    hipGraphNode_t a = fa->second, b = fb->second;
    if (hipGraphAddDependencies(parent, &a, &b, 1) != hipSuccess) return MERGE_ERROR;
  }
  return MERGE_OK;
}

struct isdf_graph_s {
  int device = 0;
  std::vector<isdf_plan> plans;
  std::vector<hipGraph_t> children;
  int merged = 0;   // systems copied node by node (the rest are child graphs)
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

isdf_status isdf_graph_destroy(isdf_graph g) {
  if (!g) return ISDF_OK;
  (void)hipSetDevice(g->device);
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (hipGraph_t c : g->children) (void)hipGraphDestroy(c);
  delete g;
  return ISDF_OK;
}

isdf_status isdf_multi_graph_create(int32_t count, const isdf_plan* plans, const void* const* psi,
                                    const double* const* energies, const double* const* omega,
                                    void* const* workspace, const size_t* ws_bytes, void* const* eps_inv,
                                    isdf_graph* out) {
  if (!out) return ISDF_E_ARG;
  *out = nullptr;
  if (count < 1 || !plans || !psi || !energies || !workspace || !ws_bytes || !eps_inv) return ISDF_E_ARG;
  for (int i = 0; i < count; ++i) {
    if (!plans[i]) return ISDF_E_ARG;
    if (plans[i]->h->device != plans[0]->h->device) return fail(plans[0]->h, ISDF_E_ARG, "plans on different devices");
    if (!plans[i]->h->stream)
      return fail(plans[i]->h, ISDF_E_ARG, "each plan's handle needs a created stream (the null stream cannot be captured)");
    TRY(plan_check(plans[i], psi[i], energies[i], omega ? omega[i] : nullptr, workspace[i], ws_bytes[i], eps_inv[i]));
    for (int j = 0; j < i; ++j)
      if (workspace[j] == workspace[i] || eps_inv[j] == eps_inv[i])
        return fail(plans[i]->h, ISDF_E_ARG, "the systems of one graph run concurrently: each needs its own workspace and output");
  }
  isdf_handle h0 = plans[0]->h;
  HIPCHK_H(h0, hipSetDevice(h0->device));
  isdf_graph g = new isdf_graph_s;
  g->device = h0->device;
  auto bail = [&](isdf_status s) { (void)isdf_graph_destroy(g); return s; };
  if (hipGraphCreate(&g->graph, 0) != hipSuccess) return bail(fail(h0, ISDF_E_DEVICE, "hipGraphCreate failed"));
  for (int i = 0; i < count; ++i) {
    // Each system is captured on its own handle's stream (its second stream joins that
    // capture directly), then its nodes and edges are copied into the parent graph with
    // no dependencies on the other systems, so the systems run concurrently when the
    // graph is launched.  A capture holding other node kinds goes in as a child graph.
    isdf_handle hi = plans[i]->h;
    hipStream_t s = hi->stream;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bail(fail(hi, ISDF_E_DEVICE, "hipStreamBeginCapture failed"));
    const isdf_status st = plan_enqueue(plans[i], psi[i], energies[i], omega ? omega[i] : nullptr, workspace[i],
                                        eps_inv[i], false);
    hipGraph_t child = nullptr;
    const hipError_t e = hipStreamEndCapture(s, &child);
    if (child) g->children.push_back(child);
    if (st != ISDF_OK) return bail(st);
    if (e != hipSuccess || !child)
      return bail(fail(hi, ISDF_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e)));
    const MergeResult m = merge_graph(g->graph, child);
    if (m == MERGE_ERROR) return bail(fail(hi, ISDF_E_DEVICE, "copying the captured nodes into the graph failed"));
    if (m == MERGE_OTHER) {
      hipGraphNode_t node;
      if (hipGraphAddChildGraphNode(&node, g->graph, nullptr, 0, child) != hipSuccess)
        return bail(fail(hi, ISDF_E_DEVICE, "hipGraphAddChildGraphNode failed"));
    } else {
      ++g->merged;
    }
    g->plans.push_back(plans[i]);
  }
  const hipError_t e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) return bail(fail(h0, ISDF_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)));
  *out = g;
  return ISDF_OK;
}

isdf_status isdf_graph_launch(isdf_graph g, void* hip_stream) {
  if (!g) return ISDF_E_ARG;
  if (hipSetDevice(g->device) != hipSuccess) return ISDF_E_DEVICE;
  hipStream_t s = (hipStream_t)hip_stream;
  if (hipGraphLaunch(g->exec, s) != hipSuccess) return ISDF_E_DEVICE;
  for (isdf_plan p : g->plans) {   // isdf_plan_sync waits for this stream
    p->last = s;
    p->last_set = true;
  }
  return ISDF_OK;
}

isdf_status isdf_plan_sync(isdf_plan pl, isdf_report* rep) {
  if (!pl) return ISDF_E_ARG;
  isdf_handle h = pl->h;
  StatusBlock hs;
  HIPCHK(hipSetDevice(h->device));
  // the stream the plan's last call was enqueued on (calls of one plan never overlap),
  // which need not be the handle's current one
  hipStream_t st = pl->last_set ? pl->last : h->stream;
  HIPCHK(hipMemcpyAsync(&hs, pl->dev, offsetof(StatusBlock, partial), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(zero_fill(pl->dev, offsetof(StatusBlock, partial), st));
  HIPCHK(hipStreamSynchronize(st));
  if (rep) for (int k = 0; k < 8; ++k) rep->stage_ms[k] = 0.0;
  if (rep && pl->tn > 0) {   // mean of each stage interval over the timed calls since the last sync
    for (int k = 0; k + 1 < pl->tmarks && k < 8; ++k) {
      double sum = 0.0;
      for (int c = 0; c < pl->tn; ++c) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pl->tev[10 * c + k], pl->tev[10 * c + k + 1]));
        sum += ms;
      }
      rep->stage_ms[k] = sum / pl->tn;
    }
  }
  pl->tn = 0;
  return report_status(h, hs, pl->P, rep);
}

static bool tune_valid(const isdf_tune* t) {
  return t && t->dft_zb >= 1 && t->dft_zb <= 64 && t->core_split_pct >= 25 && t->core_split_pct <= 200 &&
         t->gram_split >= 1 && t->gram_split <= 16 && t->wg_per_cu >= 1 && t->wg_per_cu <= 4 &&
         t->core_stream >= 0 && t->core_stream <= 2 && t->side_prio >= 0 && t->side_prio <= 1 &&
         t->dft_pipe >= 0 && t->dft_pipe <= 1;
}

isdf_status isdf_plan_set_tune(isdf_plan pl, const isdf_tune* t) {
  if (!pl) return ISDF_E_ARG;
  if (!tune_valid(t)) return fail(pl->h, ISDF_E_ARG, "tuning knob out of range");
  pl->tune.dft_zb = t->dft_zb;
  pl->tune.core_split_pct = t->core_split_pct;
  pl->tune.gram_split = t->gram_split;
  pl->tune.wg_per_cu = t->wg_per_cu;
  pl->tune.core_stream = t->core_stream;
  pl->tune.side_prio = t->side_prio;
  pl->tune.dft_pipe = t->dft_pipe;
  return ISDF_OK;
}

isdf_status isdf_plan_get_tune(isdf_plan pl, isdf_tune* t) {
  if (!pl || !t) return ISDF_E_ARG;
  t->dft_zb = pl->tune.dft_zb;
  t->core_split_pct = pl->tune.core_split_pct;
  t->gram_split = pl->tune.gram_split;
  t->wg_per_cu = pl->tune.wg_per_cu;
  t->core_stream = pl->tune.core_stream;
  t->side_prio = pl->tune.side_prio;
  t->dft_pipe = pl->tune.dft_pipe;
  t->best_ms = 0.0;
  return ISDF_OK;
}

isdf_status isdf_plan_autotune(isdf_plan pl, const void* psi, const double* energies, const double* omega,
                               void* workspace, size_t ws_bytes, void* eps_inv, int32_t reps, isdf_tune* out) {
  TRY(plan_check(pl, psi, energies, omega, workspace, ws_bytes, eps_inv));
  if (reps < 1 || reps > 100) return fail(pl->h, ISDF_E_ARG, "reps must be in [1, 100]");
  isdf_handle h = pl->h;
  HIPCHK(hipSetDevice(h->device));
  auto time_call = [&](float& ms) -> isdf_status {
    TRY(plan_enqueue(pl, psi, energies, omega, workspace, eps_inv));  // warm-up
    HIPCHK(hipEventRecord(h->ev[0], h->stream));
    for (int r = 0; r < reps; ++r) TRY(plan_enqueue(pl, psi, energies, omega, workspace, eps_inv));
    HIPCHK(hipEventRecord(h->ev[1], h->stream));
    HIPCHK(hipEventSynchronize(h->ev[1]));
    HIPCHK(hipEventElapsedTime(&ms, h->ev[0], h->ev[1]));
    ms /= (float)reps;
    return ISDF_OK;
  };
  // coordinate descent over the knobs, each over its candidate list, keeping the best so far
  // (a candidate must beat it by 0.5%)
  float best = 0.f;
  TRY(time_call(best));
  const int zbs[] = {4, 6, 8, 12, 16, 24};
  const int splits[] = {50, 100, 200};
  const int grams[] = {4, 8, 16};
  const int wpcs[] = {1, 2};
  const int cstreams[] = {0, 1, 2};
  const int prios[] = {0, 1};
  auto sweep = [&](int Tune::*knob, const int* cands, int nc) -> isdf_status {
    const int keep = pl->tune.*knob;
    int arg = keep;
    for (int i = 0; i < nc; ++i) {
      if (cands[i] == keep) continue;
      pl->tune.*knob = cands[i];
      float ms = 0.f;
      TRY(time_call(ms));
      if (ms < 0.995f * best) { best = ms; arg = cands[i]; }   // 0.5% margin against timing noise
    }
    pl->tune.*knob = arg;
    return ISDF_OK;
  };
  TRY(sweep(&Tune::dft_zb, zbs, 6));
  TRY(sweep(&Tune::core_split_pct, splits, 3));
  TRY(sweep(&Tune::gram_split, grams, 3));
  TRY(sweep(&Tune::wg_per_cu, wpcs, 2));
  TRY(sweep(&Tune::core_stream, cstreams, 3));
  TRY(sweep(&Tune::side_prio, prios, 2));
  TRY(sweep(&Tune::dft_pipe, prios, 2));
  if (out) {
    TRY(isdf_plan_get_tune(pl, out));
    out->best_ms = best;
  }
  return ISDF_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Adjoint of L = Re tr(W eps~^{-1}) (FP64).  Nothing of a forward call is kept:
// the pair products, X = V^{1/2} F Z, S, M and their inverses are recomputed,
// then the forward's steps are run backwards.  With K = (M^{-1} - U^H U)^{-1}
// and Y = U K (so that eps~^{-1} = I + U K U^H and eps~^{-1} U = U K M^{-1}):
//   T = W Y,  G_U = 2 (T + Y U^H T),  R = M^{-1} Y^H T M^{-1}    (dL/dU, dL/dM)
//   U = X S^{-1}:  Gbar = G_U S^{-1},  G_S = -U^H Gbar,  G_Z = F^H V^{1/2} Gbar
//   Z = conj(Pa) Pb:  G_Pa = conj(G_Z) Pb,  G_Pb = G_Z Pa
//   S = conj(Ga) Pb-Gram:  G_Ga = conj(G_S) Gb,  G_Gb = G_S Ga
//   M = f C diag(w) C^H:  per occupied i, U_i = R (conj(a_i) b) gives dL/da_i,
//   dL/db and dL/dw_ij = f c_ij^H R c_ij, and dL/d eps through w_ij(eps).
// Gradients follow dL/dRe + i dL/dIm; the orbital gradient is the total
// derivative with respect to each sample psi_n(r_mu).
// ---------------------------------------------------------------------------
namespace {

struct GradLayout {
  size_t pa = 0, pb = 0, t1b = 0, u = 0, y = 0, t = 0, gu = 0, gbar = 0;
  size_t ga = 0, gb = 0, s = 0, sinv = 0, m = 0, minv = 0, km = 0, p = 0, yht = 0, r = 0, tmp = 0, gs = 0;
  size_t ha = 0, hb = 0, qa = 0, q = 0, csr = 0, loss = 0, total = 0;
  int nb = 1;   // occupied states per core-backward batch (its operands reuse the pa / pb regions)
};

GradLayout grad_layout(const Problem& P, const Layout& L, int kx, int nd) {
  GradLayout G;
  size_t off = L.total;
  auto take = [&](size_t bytes) { size_t o = off; off += up(std::max<size_t>(bytes, 1)); return o; };
  const size_t cz = (size_t)(P.zrows > 0 ? P.zrows : P.nmu);   // points per chunk
  // the core backward's batches of occupied states reuse the pa / pb regions
  G.nb = (int)std::max<long>(1, std::min<long>(std::min<long>(P.nv, 64), (long)(cz * P.nr / ((size_t)P.nmu * P.nc))));
  const size_t z = 16, n2 = (size_t)P.nmu * P.nmu * z,
               tall = std::max(cz * P.nr, (size_t)G.nb * P.nmu * P.nc) * z,
               list = (size_t)P.ngg * P.nmu * z;
  G.pa = take(tall);
  G.pb = take(tall);
  G.t1b = take(cz * P.n2 * P.n1 * kx * z);
  G.u = take(list); G.y = take(list); G.t = take(list); G.gu = take(list); G.gbar = take(list);
  for (size_t* f : {&G.ga, &G.gb, &G.s, &G.sinv, &G.m, &G.minv, &G.km, &G.p, &G.yht, &G.r, &G.tmp, &G.gs,
                    &G.ha, &G.hb, &G.qa})
    *f = take(n2);
  G.q = take((size_t)P.nv * P.nc * z);
  G.csr = take((size_t)(nd + 1 + P.ngg + kx + 1 + nd) * 4);
  G.loss = take(8);
  G.total = off;
  return G;
}

// plane waves grouped by (x, y) pair, then pairs grouped by x frequency (stable order)
std::vector<int32_t> grad_csr(const DftIndex& ix, int ngg) {
  const int nd = (int)ix.d_ax.size(), kx = (int)ix.xl.size();
  std::vector<int32_t> out((size_t)nd + 1 + ngg + kx + 1 + nd, 0);
  int32_t* gd_off = out.data();
  int32_t* gd_list = gd_off + nd + 1;
  int32_t* da_off = gd_list + ngg;
  int32_t* da_list = da_off + kx + 1;
  for (int g = 0; g < ngg; ++g) ++gd_off[ix.g_d[g] + 1];
  for (int d = 0; d < nd; ++d) gd_off[d + 1] += gd_off[d];
  std::vector<int32_t> fill(gd_off, gd_off + nd);
  for (int g = 0; g < ngg; ++g) gd_list[fill[ix.g_d[g]]++] = g;
  for (int d = 0; d < nd; ++d) ++da_off[ix.d_ax[d] + 1];
  for (int a = 0; a < kx; ++a) da_off[a + 1] += da_off[a];
  std::vector<int32_t> fa(da_off, da_off + kx);
  for (int d = 0; d < nd; ++d) da_list[fa[ix.d_ax[d]]++] = d;
  return out;
}

GemmDesc gd(int M, int N, int K, const void* A, long sam, long sak, bool ca, const void* B, long sbk, long sbn,
            bool cb, void* C, long ldc, double alpha = 1.0, double beta = 0.0) {
  GemmDesc d;
  d.M = M; d.N = N; d.K = K;
  d.A = A; d.sam = sam; d.sak = sak; d.conjA = ca;
  d.B = B; d.sbk = sbk; d.sbn = sbn; d.conjB = cb;
  d.C = C; d.ldc = ldc; d.alpha = alpha; d.beta = beta;
  return d;
}

isdf_status enqueue_grad(Run& R, const GradLayout& G, const void* psi, double omega, const void* w, double* ge,
                         void* gpsi) {
  isdf_handle h = R.h;
  const Problem& P = R.P;
  const Layout& L = R.L;
  hipStream_t st = R.st;
  auto B = [&](size_t off) { return at<char>(R.ws, off); };
  const int nmu = P.nmu, nv = P.nv, nc = P.nc, ngg = P.ngg, ng = P.ng;
  const long nr = P.nr, n2 = (long)nmu * nmu;
  TRY(prepare_psi(R, psi));
  TRY(stage_points(R));
  char* pm = B(L.pm);
  const char* ps = reinterpret_cast<const char*>(R.psi);
  char* ga_out = reinterpret_cast<char*>(gpsi);
  char* gb_out = ga_out + (size_t)nv * nmu * 16;
  void* lin = B(L.lin);
  int* status = &R.sb->status;
  // split-K scratch: the Z^T region once the DFT has read it
  auto split = [&](GemmDesc d, int cap = 16) {
    d.split_ws = B(L.zt); d.split_ws_bytes = L.zt_bytes; d.max_split = cap;
    return d;
  };
  // The N_mu x Nr intermediates exist for one chunk of points [c0, c0 + cn) at a time.
  const int chunk = P.zrows > 0 ? P.zrows : nmu;
  // Pa^T, Pb^T of a chunk: Pa^T[mu][r] = sum_{i < nv} conj(psi_i(r_mu)) psi_i(r), Pb^T over the empty states
  auto pair_blocks = [&](int c0, int cn) -> isdf_status {
    HIPCHK(gemm(R.grad_big, gd(cn, (int)nr, nv, pm + (size_t)c0 * 16, 1, nmu, true, ps, nr, 1, false, B(G.pa), nr),
                st));
    HIPCHK(gemm(R.grad_big, gd(cn, (int)nr, nc, pm + ((size_t)nv * nmu + c0) * 16, 1, nmu, true,
                               ps + (size_t)nv * nr * 16, nr, 1, false, B(G.pb), nr), st));
    return ISDF_OK;
  };
  // forward, recomputed chunk by chunk: Z^T = conj(Pa^T) Pb^T, X^T = (V^{1/2} F Z)^T (rows c0..)
  TRY(dft_tables(R));
  for (int c0 = 0; c0 < nmu; c0 += chunk) {
    const int cn = std::min(chunk, nmu - c0);
    TRY(pair_blocks(c0, cn));
    HIPCHK(adj_conj_mul(B(G.pa), B(G.pb), B(L.zt), (long)cn * nr, st));
    DftPlan dp = make_plan(R);
    dp.nmu = cn;
    TRY(dft_apply(R, dp, B(L.zt), B(L.t2), L.t2_bytes, B(L.zg) + (size_t)c0 * ngg * 16, at<double>(R.ws, L.sqrtv)));
  }
  // S = conj(Ga) Gb, S^{-1}; M (with its pair weights) and M^{-1}
  HIPCHK(gemm(P64, gd(nmu, nmu, nv, pm, 1, nmu, false, pm, nmu, 1, true, B(G.ga), nmu), st));
  HIPCHK(gemm(P64, gd(nmu, nmu, nc, pm + (size_t)nv * nmu * 16, 1, nmu, false, pm + (size_t)nv * nmu * 16, nmu, 1,
                      true, B(G.gb), nmu), st));
  HIPCHK(adj_conj_mul(B(G.ga), B(G.gb), B(G.s), n2, st));
  HIPCHK(scale_z(B(G.s), B(G.sinv), n2, 1.0, st));
  HIPCHK(sweep_inverse(nmu, B(G.sinv), lin, status, st));   // -S^{-1}
  HIPCHK(scale_z(B(G.sinv), B(G.sinv), n2, -1.0, st));
  if (R.grad_big == P32 && core32_fits(nmu, nc)) {
    // mixed: the single-precision core of the forward (k-major engine, FP64 flush)
    double* wts = at<double>(R.ws, L.w);
    HIPCHK(pair_weights(R.e, nv, nc, omega, wts, st));
    const int ns = core32_splits(nmu, nv, L.nsplit);
    HIPCHK(core32_partial(nmu, nv, nc, pm, wts, B(L.part), ns, st));
    HIPCHK(core_reduce(P32, nmu, B(L.part), ns, P.f, B(G.m), B(G.minv), st));
  } else {
    TRY(stage_core(R, omega, B(G.m), B(G.minv), st));        // M, -M
  }
  HIPCHK(sweep_inverse(nmu, B(G.minv), lin, status, st));   // -(-M)^{-1} = M^{-1}
  // U = X S^{-1};  K = -(U^H U - M^{-1})^{-1}
  HIPCHK(gemm(P64, gd(ngg, nmu, nmu, B(L.zg), 1, ngg, false, B(G.sinv), nmu, 1, false, B(G.u), nmu), st));
  {
    GemmDesc d = split(gd(nmu, nmu, ngg, B(G.u), 1, nmu, true, B(G.u), nmu, 1, false, B(G.km), nmu));
    d.herm = true;
    HIPCHK(gemm(P64, d, st));
  }
  HIPCHK(axpby(B(G.km), 1.0, B(G.minv), -1.0, B(G.km), n2, st));
  HIPCHK(sweep_inverse(nmu, B(G.km), lin, status, st));      // K
  // Y = U K;  T = W Y (rows of the output list; zero below);  P = U^H T;  G_U = 2 (T + Y P)
  HIPCHK(gemm(P64, gd(ngg, nmu, nmu, B(G.u), nmu, 1, false, B(G.km), nmu, 1, false, B(G.y), nmu), st));
  if (ngg > ng) HIPCHK(zero_fill(B(G.t) + (size_t)ng * nmu * 16, (size_t)(ngg - ng) * nmu * 16, st));
  HIPCHK(gemm(P64, gd(ng, nmu, ng, w, ng, 1, false, B(G.y), nmu, 1, false, B(G.t), nmu), st));
  HIPCHK(gemm(P64, split(gd(nmu, nmu, ng, B(G.u), 1, nmu, true, B(G.t), nmu, 1, false, B(G.p), nmu)), st));
  HIPCHK(adj_loss(w, ng, ng, B(G.p), nmu, at<double>(R.ws, G.loss), st));
  HIPCHK(gemm(P64, gd(ngg, nmu, nmu, B(G.y), nmu, 1, false, B(G.p), nmu, 1, false, B(G.gu), nmu), st));
  HIPCHK(axpby(B(G.t), 2.0, B(G.gu), 2.0, B(G.gu), (long)ngg * nmu, st));
  // R = M^{-1} (Y^H T) M^{-1}
  HIPCHK(gemm(P64, split(gd(nmu, nmu, ng, B(G.y), 1, nmu, true, B(G.t), nmu, 1, false, B(G.yht), nmu)), st));
  HIPCHK(gemm(P64, gd(nmu, nmu, nmu, B(G.minv), nmu, 1, false, B(G.yht), nmu, 1, false, B(G.tmp), nmu), st));
  HIPCHK(gemm(P64, gd(nmu, nmu, nmu, B(G.tmp), nmu, 1, false, B(G.minv), nmu, 1, false, B(G.r), nmu), st));
  // Gbar = G_U S^{-1};  G_S = -U^H Gbar
  HIPCHK(gemm(P64, gd(ngg, nmu, nmu, B(G.gu), nmu, 1, false, B(G.sinv), nmu, 1, false, B(G.gbar), nmu), st));
  HIPCHK(gemm(P64, split(gd(nmu, nmu, ngg, B(G.u), 1, nmu, true, B(G.gbar), nmu, 1, false, B(G.gs), nmu, -1.0)), st));
  // Per chunk of points: G_Z^T = (F^H V^{1/2} Gbar)^T into the Z^T region, the pair blocks
  // recomputed, their cotangents in place, and the orbital gradients at the points
  // through the point side of the pair products (sum over the grid: columns c0.. of the
  // outputs) and through the grid rows that are themselves points (all columns,
  // accumulated over the chunks).
  const int* ib = R.idx;
  const int32_t* csr = reinterpret_cast<const int32_t*>(B(G.csr));
  HIPCHK(zero_fill(gpsi, (size_t)P.ns * nmu * 16, st));   // every term below accumulates
  for (int c0 = 0; c0 < nmu; c0 += chunk) {
    const int cn = std::min(chunk, nmu - c0);
    {
      AdjDft a;
      a.n0 = P.n0; a.n1 = P.n1; a.n2 = P.n2; a.nmu = cn; a.ldg = nmu; a.kx = L.kx; a.ky = L.ky; a.nd = L.nd;
      a.twx = B(L.twx); a.twy = B(L.twy); a.twz = B(L.twz);
      a.sqrtv = at<double>(R.ws, L.sqrtv);
      a.gd_off = csr; a.gd_list = csr + L.nd + 1; a.da_off = a.gd_list + ngg; a.da_list = a.da_off + L.kx + 1;
      // idx block: xl[kx] yl[ky] zl[kz] d_ax[nd] d_by[nd] g_d[ngg] g_cz[ngg] dmap
      a.d_ax = ib + L.kx + L.ky + L.kz;
      a.d_by = a.d_ax + L.nd;
      a.g_cz = ib + L.kx + L.ky + L.kz + 2 * L.nd + ngg;
      HIPCHK(adj_dft(a, B(G.gbar) + (size_t)c0 * 16, B(L.t2), B(G.t1b), B(L.zt), st));
    }
    TRY(pair_blocks(c0, cn));
    HIPCHK(adj_pair_grad(B(L.zt), B(G.pa), B(G.pb), (long)cn * nr, st));   // G_Pa^T, G_Pb^T
    HIPCHK(gemm(R.grad_big, split(gd(nv, cn, (int)nr, ps, nr, 1, false, B(G.pa), 1, nr, true,
                                     ga_out + (size_t)c0 * 16, nmu, 1.0, 1.0), 64), st));
    HIPCHK(gemm(R.grad_big, split(gd(nc, cn, (int)nr, ps + (size_t)nv * nr * 16, nr, 1, false, B(G.pb), 1, nr, true,
                                     gb_out + (size_t)c0 * 16, nmu, 1.0, 1.0), 64), st));
    HIPCHK(adj_gather_cols(B(G.pa), nr, R.mu, nmu, cn, B(G.qa), st));
    HIPCHK(gemm(P64, gd(nv, nmu, cn, pm + (size_t)c0 * 16, nmu, 1, false, B(G.qa), nmu, 1, false, ga_out, nmu, 1.0,
                        1.0), st));
    HIPCHK(adj_gather_cols(B(G.pb), nr, R.mu, nmu, cn, B(G.qa), st));
    HIPCHK(gemm(P64, gd(nc, nmu, cn, pm + ((size_t)nv * nmu + c0) * 16, nmu, 1, false, B(G.qa), nmu, 1, false, gb_out,
                        nmu, 1.0, 1.0), st));
  }
  // ... S = conj(Ga) Gb ...
  HIPCHK(adj_pair_grad(B(G.gs), B(G.ga), B(G.gb), n2, st));
  HIPCHK(adj_herm_plus(B(G.ga), B(G.ha), nmu, st));
  HIPCHK(adj_herm_plus(B(G.gb), B(G.hb), nmu, st));
  HIPCHK(gemm(P64, gd(nv, nmu, nmu, pm, nmu, 1, false, B(G.ha), 1, nmu, false, ga_out, nmu, 1.0, 1.0), st));
  HIPCHK(gemm(P64, gd(nc, nmu, nmu, pm + (size_t)nv * nmu * 16, nmu, 1, false, B(G.hb), 1, nmu, false, gb_out, nmu,
                      1.0, 1.0), st));
  // ... and the core, a batch of occupied states at a time (pair operands in pa, products in pb)
  for (int i0 = 0; i0 < nv; i0 += G.nb) {
    const int nb = std::min(G.nb, nv - i0);
    HIPCHK(adj_core_pairs(pm, nmu, nv, nc, i0, nb, B(G.pa), st));
    GemmDesc d = gd(nmu, nc, nmu, B(G.r), nmu, 1, false, B(G.pa), nc, 1, false, B(G.pb), nc);
    d.batch = nb; d.bsa = 0; d.bsb = (long)nmu * nc; d.bsc = (long)nmu * nc;
    HIPCHK(gemm(R.grad_big, d, st));   // mixed: FP32 products over the N_mu points
    HIPCHK(adj_core_grads(B(G.pb), pm, at<double>(R.ws, L.w), nmu, nv, nc, i0, nb, P.f, ga_out, B(G.q), gb_out, st));
  }
  HIPCHK(adj_energy_grad(B(G.q), R.e, nv, nc, omega, ge, st));
  return ISDF_OK;
}

}  // namespace

extern "C" {

isdf_status isdf_contour_nodes(const double* energies, int32_t nv, int32_t nc, double tol, double* out,
                               int32_t* n_out) {
  if (!energies || !out || !n_out || nv < 1 || nc < 1) return ISDF_E_ARG;
  if (!(tol > 0.0 && tol < 1e-2)) return ISDF_E_ARG;
  double vmax = -INFINITY, cmin = INFINITY;
  for (int i = 0; i < nv + nc; ++i) {
    if (!std::isfinite(energies[i])) return ISDF_E_ARG;
    if (i < nv) vmax = std::max(vmax, energies[i]);
    else cmin = std::min(cmin, energies[i]);
  }
  if (!(vmax < cmin) || energies[nv - 1] != vmax || energies[nv] != cmin) return ISDF_E_ARG;
  const std::vector<double> t = cauchy_nodes(energies, nv, nc, tol);
  std::copy(t.begin(), t.end(), out);
  *n_out = (int32_t)(t.size() / 4);
  return ISDF_OK;
}

isdf_status isdf_grad_workspace_bytes(const isdf_problem* prob, int32_t n_mu, int32_t ng, size_t* bytes) {
  if (!bytes || !prob) return ISDF_E_ARG;
  if (prob->prec == ISDF_BF16X3) return ISDF_E_UNSUPPORTED;
  isdf_problem p64 = *prob;
  p64.prec = ISDF_FP64;   // FP64 storage in both adjoint modes
  Problem P;
  isdf_status s = check_problem(nullptr, &p64, P);
  if (s != ISDF_OK) return s;
  if (n_mu < 1 || ng < 1) return ISDF_E_ARG;
  P.nmu = n_mu;
  P.ng = ng;
  P.ngg = P.full_gram ? (int)P.nr : ng;
  P.nomega = 0;
  P.zrows = grad_chunk(P);
  const int kx = std::min(P.ngg, P.n0), ky = std::min(P.ngg, P.n1), kz = std::min(P.ngg, P.n2);
  const int nd = (int)std::min<long>(P.ngg, (long)P.n0 * P.n1);
  *bytes = grad_layout(P, make_layout(P, kx, ky, kz, nd), kx, nd).total;
  return ISDF_OK;
}

isdf_status isdf_eps_inv_grad(isdf_handle h, const isdf_problem* prob, const void* psi, const double* energies,
                              const int32_t* mu_idx, int32_t n_mu, const int32_t* miller, int32_t ng, double omega,
                              const void* w, void* workspace, size_t ws_bytes, double* grad_energies,
                              void* grad_psi_mu, double* loss) {
  if (!h) return ISDF_E_ARG;
  if (!w || !grad_energies || !grad_psi_mu) return fail(h, ISDF_E_ARG, "w, grad_energies and grad_psi_mu must be non-NULL");
  if (!energies) return fail(h, ISDF_E_ARG, "energies is NULL");
  if (!miller) return fail(h, ISDF_E_ARG, "miller is NULL");
  if (!(omega >= 0.0) || !std::isfinite(omega)) return fail(h, ISDF_E_ARG, "omega must be finite and >= 0");
  Run R;
  Uploader upl;
  DftIndex ix;
  std::vector<int> idxbuf;
  if (!prob) return fail(h, ISDF_E_ARG, "problem is NULL");
  if (prob->prec == ISDF_BF16X3)
    return fail(h, ISDF_E_UNSUPPORTED, "the adjoint runs in FP64 or with FP32 grid contractions (ISDF_FP64, ISDF_FP32)");
  // the workspace holds FP64 data in both modes; ISDF_FP32 only changes the compute
  // precision of the contractions over the grid
  isdf_problem p64 = *prob;
  const bool mixed = prob->prec == ISDF_FP32;
  p64.prec = ISDF_FP64;
  TRY(setup_common(R, h, &p64, psi, mu_idx, n_mu, miller, ng, energies, 0, workspace, ws_bytes, upl, ix, idxbuf,
                   true));
  R.grad_big = mixed ? P32 : P64;
  if (R.P.core_method != 0) return fail(h, ISDF_E_UNSUPPORTED, "the adjoint differentiates the direct core (core_method = 0)");
  const GradLayout G = grad_layout(R.P, R.L, R.L.kx, R.L.nd);
  TRY(check_ws(h, workspace, ws_bytes, G.total));
  std::vector<int32_t> csr = grad_csr(ix, R.P.ngg);
  const size_t csr_bytes = csr.size() * 4;
  upl.add(G.csr, upl.hold(std::move(csr)), csr_bytes);
  HIPCHK(hipSetDevice(h->device));
  TRY(upl.run());
  TRY(clear_status(R));
  TRY(enqueue_grad(R, G, psi, omega, w, grad_energies, grad_psi_mu));
  double lval = 0.0;
  HIPCHK(hipMemcpyAsync(&lval, at<double>(workspace, G.loss), 8, hipMemcpyDeviceToHost, R.st));
  Timer none{h, false};
  TRY(finish(R, nullptr, none));
  if (loss) *loss = lval;
  return ISDF_OK;
}

}  // extern "C"
