// Library-internal definitions shared by the host runtime and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "mkpw.h"  // include/ is on the include path
#include "fft.hpp"
#include "hpsi_types.hpp"

namespace mkpw {

// C = alpha A^H B over row blocks: A rows [a_off, a_off + a_cnt) of a
// (nk, *, ld) array, likewise B; C(k) is a ldc-strided matrix, written at
// (c_roff + i, c_coff + j) and, with mirror, conj at (c_coff + j, c_roff + i).
// Null per-k pointers mean the scalar defaults a_row/a_n/... for every k.
struct GramArgs {
  const cplx<double>* A = nullptr;
  long a_kstride = 0;
  const int* a_off = nullptr;
  const int* a_cnt = nullptr;
  int a_row = 0, a_n = 0;
  const cplx<double>* B = nullptr;
  long b_kstride = 0;
  const int* b_off = nullptr;
  const int* b_cnt = nullptr;
  int b_row = 0, b_n = 0;
  int ld = 0;
  const int* npw = nullptr;
  cplx<double>* C = nullptr;
  long c_kstride = 0;
  int ldc = 0;
  const int* c_roff = nullptr;
  const int* c_coff = nullptr;
  int c_row = 0, c_col = 0;
  double alpha = 1.0;
  int mirror = 0;
  // optional: B vector j of k takes part only if b_live[k * live_kstride + j]
  // (C entries of the others are left as they were)
  const int* b_live = nullptr;
  long live_kstride = 0;
};

// Y_j = [Y_j +] alpha sum_i X_i C(c_row + i, c_col + j) for j < y_cnt, i < x_cnt.
struct CombArgs {
  const cplx<double>* X = nullptr;
  long x_kstride = 0;
  const int* x_off = nullptr;
  const int* x_cnt = nullptr;
  int x_row = 0, x_n = 0;
  cplx<double>* Y = nullptr;
  long y_kstride = 0;
  const int* y_off = nullptr;
  const int* y_cnt = nullptr;
  int y_row = 0, y_n = 0;
  int ld = 0;
  const cplx<double>* Cm = nullptr;
  long c_kstride = 0;
  int ldc = 0;
  const int* c_roff = nullptr;
  const int* c_coff = nullptr;
  int c_row = 0, c_col = 0;
  double alpha = 1.0;
  int accumulate = 0;
  // optional: output row j of k is formed only if y_live[k * live_kstride + j]
  const int* y_live = nullptr;
  long live_kstride = 0;
};

struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
};

}  // namespace mkpw

struct pw_ctx {
  int device = -1;
  bool host_only = true;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  // options
  int64_t hbm_budget = 0;  // 0 = no budget
  int64_t trace = 0;
  int64_t dav_basis_factor = 4;
  int64_t hpsi_variant = 0;  // 0 = autotuned, else the kernel variant (1, 2)
  int64_t hpsi_slab = 0;     // 0 = autotuned, else z planes per slab
  int64_t hpsi_threads = 0;  // 0 = autotuned, else work-items per workgroup
  int64_t tune_log = 0;      // print the autotuning timings to stderr
  int64_t solver_graph = 1;  // replay one solver iteration as a captured HIP graph
  int64_t mixed_refine = 1;  // mixed-precision Davidson: refine in FP64 after the complex64 phase
  int64_t mixed_switch_rtol_e7 = 2000;  // mixed Davidson: residual norm ending the complex64 phase, 1e-7 units
  int64_t cg_switch_digits = 10;  // mixed-precision CG: leave complex64 once |rho| fell by 10^-digits
  int64_t dav_nconv = 0;          // Davidson: bands that must converge (0: all; the rest are buffer bands)
  // statistics of the last solver call: iterations run, and k-band rows H was
  // applied to (each (k, vector) row counted once per application)
  int64_t last_iterations = 0, last_hpsi_kbands = 0, last_graph_replays = 0;
  int last_hpsi_variant = 0, last_hpsi_slab = 0, last_hpsi_threads = 0;  // shape of the last H|psi> launch

  // crystal and basis
  bool have_lattice = false, have_cutoff = false, have_k = false, have_v = false, have_proj = false;
  double lat[9] = {0}, rec[9] = {0};
  double ecut_ry = 0;
  int fft[3] = {0, 0, 0};
  int nk = 0, npwx = 0;
  std::vector<double> kcart;
  std::vector<int> npw, nstick;
  std::vector<int32_t> miller;  // nk * npwx * 3
  std::vector<int> mlo, mhi;     // nk * 3: smallest and largest Miller index of each k's sphere per axis
  std::vector<double> kin;      // nk * npwx
  std::vector<int> gmap;        // nk * npwx
  std::vector<short> sof;       // nk * wx * wy
  int wx = 0, wy = 0, wz = 0, smax = 0;

  // page-locked host memory for the solvers' small per-iteration copies,
  // grown on demand and freed with the context
  void* pin = nullptr;
  size_t pin_cap = 0;

  // device copies
  std::vector<mkpw::DevMem> owned;
  int* d_npw = nullptr;
  int* d_nstick = nullptr;
  int* d_gmap = nullptr;
  short* d_sof = nullptr;
  double* d_kin = nullptr;
  int* d_mkey = nullptr;    // (nk, npwx) packed Miller index ((m1+512)<<20 | (m2+512)<<10 | (m3+512))
  int* d_lexperm = nullptr; // (nk, npwx) plane-wave indices of each sphere in lexicographic Miller order
  double v0 = 0.0;          // mean of V(r): its G = 0 Fourier coefficient (Ha)
  double* d_v64 = nullptr;  // V(r) / N_r
  float* d_v32 = nullptr;
  void* d_vperm64 = nullptr;  // V/N_r permuted for the kernel's slab width
  void* d_vperm32 = nullptr;
  int vperm_l3c64 = 0, vperm_l3c32 = 0;
  void* d_xtaps64 = nullptr;  // x-line convolution taps of V/N_r for a window capacity
  void* d_xtaps32 = nullptr;
  int xtaps_wc64 = 0, xtaps_wc32 = 0;
  int nproj = 0;
  void* d_beta64 = nullptr;  // (nk, nproj, npwx) complex double
  void* d_beta32 = nullptr;  // complex float
  void* d_dij64 = nullptr;   // (nproj, nproj) complex double
  void* d_dij32 = nullptr;
  std::vector<double> dij;   // host copy, complex interleaved
  bool have_q = false;       // overlap S = 1 + sum_pq |beta_p> q_pq <beta_q| set
  void* d_q64 = nullptr;     // (nproj, nproj) complex double
  void* d_q32 = nullptr;     // complex float
  std::vector<double> qij;   // host copy, complex interleaved

  mkpw::KTables tables() const;
};

namespace mkpw {

pw_status set_err(pw_ctx* c, pw_status s, const std::string& msg);
pw_status dev_alloc(pw_ctx* c, size_t bytes, void** out);
void dev_free(pw_ctx* c, void* p);
// c->pin with at least `bytes` (the context's stream is synchronised first)
pw_status host_pinned(pw_ctx* c, size_t bytes, void** out);

// H|psi> over the selected vectors (kernels in hpsi.hip). psi/hpsi are
// complex double (prec = PW_FP64) or complex float (PW_MIXED).
// vscratch: see launch_shape (hpsi_kernel.hpp); null for the context's own
// permuted potential.
pw_status launch_hpsi(pw_ctx* c, pw_prec prec, const VecSel& sel, const void* psi, void* hpsi,
                      hipStream_t stream, void* vscratch = nullptr);
pw_status hpsi_scratch_init(pw_ctx* c);
bool hpsi_supported(int n1, int n2, int n3);

// S|psi> = psi + sum_pq beta_p q_pq <beta_q|psi> over the selected vectors
// (spsi.hip; S = 1 when no overlap is set).  Without `scale` it writes
// out = S psi (padding zero); with `scale` ([nk * sel.nvec], indexed by k and
// the row's position in the selection) it accumulates
// out += mult * scale[k * sel.nvec + r] * S psi on the plane waves of k.
pw_status launch_spsi(pw_ctx* c, pw_prec prec, const VecSel& sel, const void* psi, void* out, const double* scale,
                      double mult, hipStream_t st);

pw_status check_launch(pw_ctx* c, const char* what, hipStream_t st);
// thread-safe, once-per-kernel raise of the dynamic LDS limit (needed above 64 KiB)
pw_status ensure_lds_limit(pw_ctx* c, const void* kernel, size_t lds);
// a kernel's registers per lane and scratch bytes per lane, read once per
// process under the lock that also covers ensure_lds_limit; false on failure
bool kernel_resources(const void* kernel, int* regs, size_t* scratch);
pw_status launch_gram(pw_ctx* c, const GramArgs& a, int ni_max, int nj_max, hipStream_t st);
pw_status launch_combine(pw_ctx* c, const CombArgs& a, int ni_max, hipStream_t st);
pw_status launch_trmm(pw_ctx* c, cplx<double>* Y, long y_kstride, const int* y_off, const int* y_cnt,
                      const cplx<double>* M, long m_kstride, int ldm, hipStream_t st);
// (with `live`, [nk * nvec], row v of k is converted only if live[k * nvec + v])
pw_status launch_to_c64(pw_ctx* c, const cplx<double>* src, long s_kstride, const int* s_off, cplx<float>* dst,
                        long d_kstride, const int* d_off, const int* cnt, int nvec, hipStream_t st,
                        const int* live = nullptr);
pw_status launch_to_c128(pw_ctx* c, const cplx<float>* src, long s_kstride, const int* s_off, cplx<double>* dst,
                         long d_kstride, const int* d_off, const int* cnt, int nvec, hipStream_t st,
                         const int* live = nullptr);

// Hermitian eigensolver (Householder tridiagonalization, bisection and inverse
// iteration, one workgroup per k, LDS):
// for each k with n[k] > 0, the n x n matrix A(k) (lda-strided) -> the lowest
// nev eigenvalues (ascending) into w[k*nev..] and their eigenvectors as the
// columns of V(k) (n x nev, ldv-strided).  n <= 64.
pw_status launch_heev(pw_ctx* c, const cplx<double>* A, long a_kstride, int lda, const int* n, int nmax, int nev,
                      double* w, cplx<double>* V, long v_kstride, int ldv, hipStream_t st);
// Cholesky of the Hermitian positive definite S(k) (n[k] x n[k], <= 32) and
// M(k) = L^-H (upper triangular) so that Y M has orthonormal rows when
// S = Y Y^H; info[k] = 0 on success, 1 when S is not numerically positive.
pw_status launch_chol_inv(pw_ctx* c, const cplx<double>* S, long s_kstride, int lds, const int* n, cplx<double>* M,
                          long m_kstride, int ldm, int* info, hipStream_t st);

}  // namespace mkpw
