// Host-side launch interface between the C-ABI layer (api.hip) and the kernels.
// Every launcher enqueues on `st` and returns the launch status.  Matrices are
// row-major complex (interleaved) unless stated otherwise; "z" = complex128,
// "c" = complex64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace isdf {

enum Prec { P64 = 0, P32 = 1, PBF3 = 2 };

// ----- generic complex GEMM:  C = alpha * diag(rs) * op(A) op(B) + beta * C + diag_add * I
struct GemmDesc {
  int M = 0, N = 0, K = 0;
  const void* A = nullptr; long sam = 0, sak = 0; bool conjA = false; bool a32 = false;
  const void* B = nullptr; long sbk = 0, sbn = 0; bool conjB = false; bool b32 = false;
  void* C = nullptr; long ldc = 0; bool c32 = false;
  double alpha = 1.0, beta = 0.0, diag_add = 0.0;
  const double* row_scale = nullptr;  // device, length M, optional
  bool herm = false;                  // only lower tiles; upper mirrored as conj
  // optional split-K scratch (device): when set, K is split across workgroups and the
  // partial sums are reduced in a fixed order by a second kernel
  void* split_ws = nullptr; size_t split_ws_bytes = 0;
  // batch of independent products (no split-K): operand / result strides in complex elements
  int batch = 1; long bsa = 0, bsb = 0, bsc = 0;
  int max_split = 16;  // cap on the split-K factor (a tuning knob)
};
// Compute precision: P64 -> f64 MFMA; P32 -> f32 MFMA.
hipError_t gemm(Prec compute, const GemmDesc& d, hipStream_t st);
// Single-precision complex GEMM with k-major operands, full tiles only
// (M % 128 = N % 64 = K % 16 = 0, even leading dimensions, 16-byte aligned bases;
// otherwise hipErrorNotSupported and nothing is launched):
//   A(m, k) = A[k lda + m], B(k, n) = B[k ldb + n] (complex64, optionally conjugated)
//   herm_identity = false: C[m][n] = alpha (A B)[m][n], complex64, ldc
//   herm_identity = true (M = N): C = diag I + alpha A B, complex128, lower triangle
//     computed and mirrored (the product must be Hermitian), diagonal real
// tail_ws (optional, tail_bytes >= gemm32_tail_bytes(wg_per_cu)): scratch for the
// K slices of the tiles left over after whole rounds (see gemm32.hip)
hipError_t gemm32_kmajor(int M, int N, int K, const void* A, long lda, bool conjA, const void* B, long ldb,
                         bool conjB, void* C, long ldc, bool herm_identity, double alpha, hipStream_t st,
                         int wg_per_cu = 1, void* tail_ws = nullptr, size_t tail_bytes = 0, double diag = 1.0);
// dst[c][r] = src[r lds + c] (complex64, rows x cols in, cols x rows out)
hipError_t transpose_c32(int rows, int cols, const void* src, long lds, void* dst, hipStream_t st);
size_t gemm32_tail_bytes(int wg_per_cu);
bool gemm32_fits(int M, int N, int K, const void* A, long lda, const void* B, long ldb);

// ----- orbital pair Gram (step 1):  out[mu][c] = conj(Pv(mu, c)) * Qc(mu, c)
//   Pv(mu, c) = sum_{i < nv} conj(pm[i][mu]) b[i][c],  Qc(mu, c) = sum_{b0 <= j < b0 + ns - nv} conj(pm[j][mu]) b[j][c]
//   pm: [states][ldp] (orbitals at the points), b: [states][ldb] (orbitals on the grid, complex128).
//   The second state range starts at b0 (default nv: the empty states after the occupied
//   ones); the ranges may overlap (the self-energy pair sets: occupied x all, all x all).
//   P64: pm complex128, in32 = out32 = false, out complex128.  P32: pm complex64 (in32 = true),
//   b rounded to FP32 as it is staged, out complex64 (out32 = true).
hipError_t zpair(Prec compute, int M, int N, int nv, int ns, const void* pm, long ldp, const void* b,
                 long ldb, bool in32, void* out, long ldo, bool out32, hipStream_t st, int wg_per_cu = 1,
                 int b0 = -1);

// ----- core (step 2): partial sums over occupied ranges of
//   M(mu, nu) = sum_{i, j} conj(a_i(mu)) b_j(mu) w_ij a_i(nu) conj(b_j(nu))
// pm: [ns][ldp] complex128; w: [nv][nc] double; part: nsplit x nmu x nmu complex (f64 or f32 per compute)
int core_splits(int nmu, int nv);
// Single-precision core on the k-major engine (core32.hip): FP64 point samples in,
// complex64 partial sums out (as core_partial); needs nmu % 128 == 0, nc % 32 == 0.
bool core32_fits(int nmu, int nc);
int core32_splits(int nmu, int nv, int max_split);
hipError_t core32_partial(int nmu, int nv, int nc, const void* pm, const double* w, void* part, int nsplit,
                          hipStream_t st, int batch = 1);
// batch > 1: w holds batch weight sets [b][nv * nc], part [b][nsplit][nmu * nmu]
hipError_t core_partial(Prec compute, int nmu, int nv, int nc, const void* pm, long ldp,
                        const double* w, void* part, int nsplit, hipStream_t st, int batch = 1);
// M_out = scale * sum_s part[s]; writes complex128 (and optionally -M into negm)
hipError_t core_reduce(Prec compute, int nmu, const void* part, int nsplit, double scale, void* m_out,
                       void* negm_out, hipStream_t st, int batch = 1);

// ----- small FP64 dense algebra, row-major n x n complex128, ld = n
// In-place Hermitian positive definite sweep: A <- -A^{-1}.  scratch: linalg_scratch_bytes(n).
// first_done (batch 1): the first pivot block's inverse is already in scratch (form_h with
// this scratch made it), so no separate launch forms it.
hipError_t sweep_inverse(int n, void* a, void* scratch, int* status, hipStream_t st, int batch = 1,
                         bool prio = true, bool first_done = false);
size_t linalg_scratch_bytes(int n);

// ----- grid / plane-wave helpers
hipError_t widen_real(const double* src, void* dst, long count, hipStream_t st);
hipError_t gather_points(const void* psi, long nr, int ns, const int* mu, int nmu, void* pm,
                         hipStream_t st);
hipError_t pair_weights(const double* e, int nv, int nc, double omega, double* w, hipStream_t st);
// sets `bit` in *status unless the energies are finite with max(e[0:nv]) < min(e[nv:nv+nc])
hipError_t check_gap(const double* e, int nv, int nc, int* status, int bit, hipStream_t st);
hipError_t coulomb_sqrt(const int* miller, int ng, const double* recip /*3x3 rows*/, double v_scale,
                        double* sqrtv, hipStream_t st);
// DFT tables: twiddles tw[a][x] = exp(-2 pi i m_a x / n) / sqrt(n) for a list of m values
hipError_t dft_twiddles(const int* mlist, int nm, int n, bool f32, void* tw, hipStream_t st);
struct DftPlan {
  int n0, n1, n2, nmu, ng;
  int kx, ky, nd, kz;      // kept x- and y-frequencies, distinct (x, y) pairs, kept z-frequencies
  const void* twx;         // kx x n0
  const void* twy;         // ky x n1 (indexed by d_y)
  const void* twz;         // kz x n2
  const int* d_ax;         // nd: index into twx list for pair d
  const int* d_by;         // nd: index into twy list for pair d
  const int* g_d;          // ng: pair index of plane wave g
  const int* g_cz;         // ng: index into twz list of plane wave g
  const int* dmap;         // kx x ky: pair index d of (x-frequency a, y-frequency b), or -1
  const int* gd_off;       // nd + 1: plane waves of pair d are gd_list[gd_off[d] .. gd_off[d + 1])
  const int* gd_list;      // ng
  int zb = 8;              // z-planes per workgroup of dft_xy (a tuning knob)
  int pipe = 1;            // single precision: the warp-specialised fused pass where its shape fits
};
// zt: [nmu][n2][n1][n0] (compute type) -> t2: [nmu][nd][n2] -> zg: [nmu][ng] (times scale[g] if given)
hipError_t dft_xy(Prec compute, const DftPlan& p, const void* zt, void* t2, hipStream_t st);
// All three stages in one pass (kx, ky <= 32 and few plane waves per thread):
// zt -> zg (times scale[g] if given), with per-point partial sums in `part` (at
// most DFT_MAX_ZBLOCKS x nmu x ng elements).  hipErrorNotSupported when the shape
// or `part_bytes` does not fit (the caller then runs dft_xy + dft_z).
constexpr int DFT_MAX_ZBLOCKS = 8;
bool dft_fused_fits(Prec compute, const DftPlan& p);
hipError_t dft_fused(Prec compute, const DftPlan& p, const void* zt, void* part, size_t part_bytes, void* zg,
                     const double* scale, hipStream_t st);
hipError_t dft_z(Prec compute, const DftPlan& p, const void* t2, void* zg, const double* scale,
                 hipStream_t st);
bool dft_supported(int n0, int n1, int n2, int kx, int ky, Prec compute);  // LDS fits

hipError_t conj_transpose(int n, const void* a, void* at, hipStream_t st);   // at = a^H (z64)
hipError_t convert_z(const void* src, bool src32, void* dst, bool dst32, long count, hipStream_t st);

// ----- BF16x3 split precision (bf3.hip): operands split into bf16 hi / lo planes
inline int bf3_pad(int n) { return (n + 15) / 16 * 16; }           // states per phase, whole k tiles
inline long bf3_rpad(long nr) { return (nr + 127) / 128 * 128; }   // grid rows, whole row blocks
inline int bf3_npad(int nmu) { return (nmu + 63) / 64 * 64; }       // points, whole point blocks
size_t bf3_rows_bytes(long nr, int nv, int nc);
size_t bf3_points_bytes(int nmu, int nv, int nc);
// psi: complex128 [state][row], row stride ld; planes: bf3_rows_bytes
hipError_t bf3_split_rows(const void* psi, long ld, long nr, int nv, int nc, void* planes, hipStream_t st);
// pm: complex128 [state][point], row stride ld; planes: bf3_points_bytes
hipError_t bf3_split_points(const void* pm, long ld, int nmu, int nv, int nc, void* planes, hipStream_t st);
// out[mu][r] = conj(Pv) Qc (complex64, row stride ldo) from the split planes
hipError_t zpair_bf3(long nr, int nmu, int nv, int nc, const void* rows, const void* points, void* out, long ldo,
                     hipStream_t st);
// BF16x3 core (core_bf3.hip): A planes of the empty states at the points (split once per
// build into planes of core_bf3_plane_bytes), then partial sums as core_partial.  Needs
// nmu % 128 == 0 and nc % 16 == 0.
bool core_bf3_fits(int nmu, int nc);
size_t core_bf3_plane_bytes(int nmu, int nc);
hipError_t core_bf3_split(int nmu, int nv, int nc, const void* pm, void* planes, hipStream_t st);
hipError_t core_bf3_partial(int nmu, int nv, int nc, const void* pm, const void* planes, const double* w,
                            void* part, int nsplit, hipStream_t st, int batch = 1);
hipError_t axpby(const void* A, double a, const void* B, double b, void* C, long count, hipStream_t st);  // z64

// ----- contour-integral core (cauchy.hip), complex128 storage
// ops[kk][n][nu] = (n < nv ? pm[n][nu] : conj(pm[n][nu])) / (lam[k0 + kk] - e[n]), complex64 if ops32
hipError_t cauchy_scale(const void* pm, const double* e, const void* lam, int nmu, int nv, int ns, int k0, int kc,
                        void* ops, bool ops32, hipStream_t st);
// s += sum_kk w[k0 + kk] av[kk] (.) ac[kk]  (nmu x nmu, fixed node order; products complex64 if prod32)
hipError_t cauchy_accum(const void* av, const void* ac, bool prod32, const void* w, int k0, int kc, int nmu, void* s,
                        hipStream_t st);
// m = f / (2 pi i) (s - s^H), negm = -m (either may be null)
hipError_t cauchy_finish(const void* s, int nmu, double f, void* m, void* negm, hipStream_t st);

// ----- adjoint of L = Re tr(W eps~^{-1}) (adjoint.hip), complex128 throughout
hipError_t adj_conj_mul(const void* x, const void* y, void* out, long n, hipStream_t st);   // out = conj(x) y
hipError_t adj_pair_grad(const void* g, void* p, void* q, long n, hipStream_t st);        // p <- conj(g) q, q <- g p
hipError_t adj_herm_plus(const void* g, void* h, int n, hipStream_t st);                   // h = g + g^H
hipError_t adj_gather_cols(const void* src, long ld, const int* idx, int nv, int rows, void* out, hipStream_t st);
// adjoint of the pruned DFT: gz[mu][r] = sum_g conj(F(g, r)) sqrtv[g] gbar[g][mu]
struct AdjDft {
  int n0 = 0, n1 = 0, n2 = 0, nmu = 0, kx = 0, ky = 0, nd = 0;   // nmu: columns of gbar transformed
  long ldg = 0;                                          // gbar: [g][ldg] complex128
  const void* twx = nullptr; const void* twy = nullptr; const void* twz = nullptr;   // forward tables
  const double* sqrtv = nullptr;
  const int* gd_off = nullptr; const int* gd_list = nullptr;   // plane waves grouped by (x, y) pair
  const int* g_cz = nullptr;                                   // plane wave -> z-frequency index
  const int* da_off = nullptr; const int* da_list = nullptr;   // pairs grouped by x frequency
  const int* d_ax = nullptr;                                   // pair -> x-frequency index
  const int* d_by = nullptr;                                   // pair -> y-frequency index
};
hipError_t adj_dft(const AdjDft& a, const void* gbar, void* t2b, void* t1b, void* gz, hipStream_t st);
hipError_t adj_core_pairs(const void* pm, int nmu, int nv, int nc, int i0, int nb, void* cb, hipStream_t st);
hipError_t adj_core_grads(const void* ub, const void* pm, const double* w, int nmu, int nv, int nc, int i0, int nb,
                          double f, void* ga, void* q, void* gb, hipStream_t st);
hipError_t adj_energy_grad(const void* q, const double* e, int nv, int nc, double omega, double* ge, hipStream_t st);
hipError_t adj_loss(const void* w, int ng, long ldw, const void* p, int n, double* out, hipStream_t st);
hipError_t zero_fill(void* p, size_t bytes, hipStream_t st);  // kernel clear, bytes % 4 == 0
// ----- self-energy reductions (sigma.hip), complex128
hipError_t mul_z(const void* a, const void* b, void* c, long count, hipStream_t st);   // c = a (.) b
// out[n] = coef Re sum_mu conj(pm[n][mu]) e[mu][n], n < ns (pm: [ns][nmu], e: [nmu][ns])
hipError_t sigma_diag(const void* pm, const void* e, int nmu, int ns, double coef, double* out, hipStream_t st);
hipError_t scale_z(const void* src, void* dst, long count, double alpha, hipStream_t st);  // z64
// out[0] += ||a||_F^2 over count complex128, deterministic (single pass of block partials)
// ||a||_F^2 of count complex128 into out; with copy32, a also goes to complex64 there (same pass)
hipError_t frob2(const void* a, long count, double* partial /*>= 1024*/, double* out, hipStream_t st,
                 void* copy32 = nullptr);
hipError_t diag_min(const void* a, int n, double* out, hipStream_t st, int batch = 1);
// H = G - K (n x n complex128), ||H||_F^2 into h2 and min Re diag(H) into hmin; partial: >= 1024 doubles
// With sweep_scratch (the scratch of the sweep_inverse(n, H, ...) that follows, batch 1), the
// same launch also inverts H's first pivot block into it (status: bit 1 if not positive
// definite); call that sweep with first_done.
hipError_t form_h(const void* G, const void* K, void* H, int n, double* partial, double* h2, double* hmin,
                  hipStream_t st, void* sweep_scratch = nullptr, int* status = nullptr);
// H[b] = G - K[b] for b < batch (complex128, n2 elements each)
hipError_t sub_bcast(const void* G, const void* K, void* H, long n2, int batch, hipStream_t st);

}  // namespace isdf
