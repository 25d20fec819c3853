// Batched block-Davidson eigensolver over many k-points (Sec. 2.1; the
// many-k form of Sec. 3, Algorithm new_gpu: every k-point of the context
// advances in the same launches and stops on its own).
//
// The problem is H psi = eps S psi (S = 1 without an overlap).  Per k-point
// the basis is kept S-orthonormal in FP64, so the reduced problem
// (H~ - eps S~) v = 0 of Sec. 2.1 has S~ = I and is solved by the batched
// Hermitian eigensolver.  SV = S V is carried along with V (updated by the
// same row operations), so S is applied once per new vector.  One iteration:
//   X = V C, HX = HV C, SX = S X             Ritz vectors of the current basis
//   R = HX - theta SX, |R|                   residuals
//   converged band: |theta - theta_prev| < tol and |R| < rtol
//   T = R / (H_diag - theta S_diag)          correction vectors for the others
//                                            (Sec. 2.1, with a 1e-2 Ha guard
//                                            on the denominator)
//   if N_base + N_nc > N_max:  restart from the Ritz vectors (V = X, ...)
//   ST = S T; T <- T - V (SV^H T) twice, normalise, Cholesky-orthonormalise
//   in the S inner product twice
//   HT = H T  (pw_h_psi kernels on the new rows only; complex64 in the
//              mixed-precision phase)
//   extend H~ by V^H HT, diagonalise -> theta, C
// The mixed-precision solve runs this loop with H applied in complex64 until
// the eigenvalues settle at the FP32 level, then restarts from its Ritz
// vectors with H applied in FP64 and iterates to the requested tolerance.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <limits>
#include <string>
#include <vector>

#include "host_util.hpp"
#include "internal.hpp"

namespace mkpw {

using cd = cplx<double>;

namespace {

__device__ __forceinline__ double block_sum(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  return s;
}

// H_diag(k, G) = |k+G|^2/2 + V~(0) + Re sum_pq beta_p D_pq beta_q^*
// S_diag(k, G) = 1 + Re sum_pq beta_p q_pq beta_q^*   (qij null: 1)
__global__ void hdiag_kernel(const int* npw, int npwx, const double* kin, double v0, int nproj, const cd* beta,
                             const cd* dij, const cd* qij, double* hd, double* sd) {
  const int k = blockIdx.y;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= npwx) return;
  double h = 0.0, s = 1.0;
  if (g < npw[k]) {
    h = kin[(long)k * npwx + g] + v0;
    const cd* b = beta + (long)k * nproj * npwx;
    for (int p = 0; p < nproj; ++p) {
      cd bp = b[(long)p * npwx + g];
      for (int q = 0; q < nproj; ++q) {
        cd bq = b[(long)q * npwx + g];
        cd d = dij[p * nproj + q];
        // Re(bp * d * conj(bq))
        double tr = bp.x * d.x - bp.y * d.y, ti = bp.x * d.y + bp.y * d.x;
        h += tr * bq.x + ti * bq.y;
        if (qij) {
          cd e = qij[p * nproj + q];
          double ur = bp.x * e.x - bp.y * e.y, ui = bp.x * e.y + bp.y * e.x;
          s += ur * bq.x + ui * bq.y;
        }
      }
    }
  }
  hd[(long)k * npwx + g] = h;
  sd[(long)k * npwx + g] = s;
}

// residuals and corrections of the nbnd Ritz pairs of every active k
__global__ __launch_bounds__(256) void resid_kernel(const cd* SX, const cd* HX, const double* theta, const int* active,
                                                    const double* hd, const double* sd, const int* npw, int npwx,
                                                    int nbnd, cd* T, cd* R, double* rnorm) {
  const int k = blockIdx.y, j = blockIdx.x;
  if (!active[k]) return;
  __shared__ double red[4];
  const long row = ((long)k * nbnd + j) * npwx;
  const double th = theta[(long)k * nbnd + j];
  const int n = npw[k];
  double s = 0.0;
  for (int g = threadIdx.x; g < npwx; g += 256) {
    cd t = {0.0, 0.0};
    if (g < n) {
      cd x = SX[row + g], hx = HX[row + g];
      cd r = {hx.x - th * x.x, hx.y - th * x.y};
      s += r.x * r.x + r.y * r.y;
      double den = hd[(long)k * npwx + g] - th * sd[(long)k * npwx + g];
      if (fabs(den) < 1e-2) den = den < 0 ? -1e-2 : 1e-2;
      t = {r.x / den, r.y / den};
      R[row + g] = r;
    } else {
      R[row + g] = {0.0, 0.0};
    }
    T[row + g] = t;
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) rnorm[(long)k * nbnd + j] = sqrt(s);
}

// V[nb + r] = T[map[r]] for r < nnc (only the slots with mask != 0 when a mask is given)
__global__ void gather_rows_kernel(const cd* T, int nbnd, cd* V, int nbmax, const int* nb, const int* nnc,
                                   const int* map, int npwx, const int* mask) {
  const int k = blockIdx.y, r = blockIdx.z;
  if (r >= nnc[k]) return;
  if (mask && !mask[(long)k * nbnd + r]) return;
  const cd* src = T + ((long)k * nbnd + map[(long)k * nbnd + r]) * npwx;
  cd* dst = V + ((long)k * nbmax + nb[k] + r) * npwx;
  for (int g = blockIdx.x * blockDim.x + threadIdx.x; g < npwx; g += gridDim.x * blockDim.x) dst[g] = src[g];
}

// restart: V[0:nbnd] = X, HV[0:nbnd] = HX (and SV = SX when SX is given), H~ = diag(theta)
__global__ void restart_kernel(const int* flag, const cd* X, const cd* HX, const cd* SX, cd* V, cd* HV, cd* SV,
                               int nbnd, int nbmax, int npwx, cd* Hr, const double* theta) {
  const int k = blockIdx.y;
  if (!flag[k]) return;
  const long n = (long)nbnd * npwx;
  const cd* xs = X + (long)k * n;
  const cd* hs = HX + (long)k * n;
  cd* vd = V + (long)k * nbmax * npwx;
  cd* hd = HV + (long)k * nbmax * npwx;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) {
    vd[e] = xs[e];
    hd[e] = hs[e];
    if (SX) SV[(long)k * nbmax * npwx + e] = SX[(long)k * n + e];
  }
  if (blockIdx.x == 0) {
    cd* h = Hr + (long)k * nbmax * nbmax;
    for (int e = threadIdx.x; e < nbmax * nbmax; e += blockDim.x) {
      int i = e / nbmax, jj = e % nbmax;
      h[e] = {(i == jj && i < nbnd) ? theta[(long)k * nbnd + i] : 0.0, 0.0};
    }
  }
}

// norms of rows [off, off + cnt) of each k into nrm[k * ldn + r]; scaled to unit
// norm when scale != 0, the same rows of V2 (if given) by the same factor
__global__ __launch_bounds__(256) void normalize_rows_kernel(cd* V, cd* V2, long kstride, const int* off,
                                                             const int* cnt, int npwx, double* nrm, int ldn,
                                                             int scale) {
  const int k = blockIdx.y, r = blockIdx.x;
  if (r >= cnt[k]) return;
  __shared__ double red[4];
  cd* v = V + (long)k * kstride + (long)(off[k] + r) * npwx;
  double s = 0.0;
  for (int g = threadIdx.x; g < npwx; g += 256) s += v[g].x * v[g].x + v[g].y * v[g].y;
  s = block_sum(s, red);
  if (threadIdx.x == 0 && nrm) nrm[(long)k * ldn + r] = sqrt(s);
  if (!scale) return;
  const double f = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
  for (int g = threadIdx.x; g < npwx; g += 256) v[g] = {v[g].x * f, v[g].y * f};
  if (V2) {
    cd* w = V2 + (long)k * kstride + (long)(off[k] + r) * npwx;
    for (int g = threadIdx.x; g < npwx; g += 256) w[g] = {w[g].x * f, w[g].y * f};
  }
}

// copy rows [0, nbnd) of src (nbnd rows per k) into rows [0, nbnd) of dst (dst_rows per k)
__global__ void copy_rows_kernel(const cd* src, int src_rows, cd* dst, int dst_rows, int nbnd, int npwx) {
  const int k = blockIdx.y;
  const long n = (long)nbnd * npwx;
  const cd* s = src + (long)k * src_rows * npwx;
  cd* d = dst + (long)k * dst_rows * npwx;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) d[e] = s[e];
}

template <class T>
__global__ void fill_kernel(T* p, long n, T v) {
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < n; e += (long)gridDim.x * blockDim.x) p[e] = v;
}

// ---- per-k bookkeeping, decided on the device so that an iteration needs no
//      host round trip (and can be replayed as a captured graph)

// Every k restarts its basis from nothing with nbnd new vectors to
// orthonormalise: nb = 0, nnc = nbnd, active, no previous eigenvalues.
__global__ void dav_reset_kernel(int nk, int nbnd, int* nb, int* nnc, int* active, int* force_restart,
                                 double* th_old) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  nb[k] = 0;
  nnc[k] = nbnd;
  active[k] = 1;
  force_restart[k] = 0;
  for (int j = 0; j < nbnd; ++j) th_old[(long)k * nbnd + j] = HUGE_VAL;
}

// After the residuals (Sec. 2.1): a band needs a correction unless its
// eigenvalue moved by less than etol and its residual norm is below rtol; a
// k none of whose lowest nconv bands needs one is converged and frozen (with
// nconv < nbnd the bands above are buffer bands: corrected while the k runs,
// which speeds up the bands below when the spectrum is nearly degenerate at
// the top of the block, but not waited for).  The bands that need one are
// listed in map[k][0 .. nnc), and a k whose basis would outgrow nbmax (or
// whose last block was dropped) restarts from its Ritz vectors (flag, nb =
// nbnd).  One wave per k, lane j = band j.
__global__ __launch_bounds__(64) void dav_decide_kernel(int nbnd, int nconv, int nbmax, double etol, double rtol,
                                                        const double* __restrict__ theta, const double* __restrict__ rn,
                                                        double* th_old, int* active, int* nb, int* nnc, int* flag,
                                                        int* map, int* force_restart, int* iters, int* nactive) {
  const int k = blockIdx.x, j = threadIdx.x;
  if (!active[k]) {
    if (j == 0) {
      nnc[k] = 0;
      flag[k] = 0;
    }
    return;
  }
  const long o = (long)k * nbnd + j;
  bool todo = false;
  if (j < nbnd) {
    const double th = theta[o];
    todo = !(fabs(th - th_old[o]) < etol && rn[o] < rtol);
    th_old[o] = th;
  }
  const unsigned long long m = __ballot(todo);
  if (todo) map[(long)k * nbnd + __popcll(m & ((1ull << j) - 1ull))] = j;
  if (j == 0) {
    const int cnt = __popcll(m);
    // the k is done once its lowest nconv bands are (buffer bands above them
    // are corrected while it runs, but need not converge)
    const unsigned long long need = nconv >= 64 ? ~0ull : (1ull << nconv) - 1ull;
    iters[k] += 1;
    if ((m & need) == 0) {
      active[k] = 0;
      nnc[k] = 0;
      flag[k] = 0;
    } else {
      atomicAdd(nactive, 1);
      nnc[k] = cnt;
      const int f = (nb[k] + cnt > nbmax) || force_restart[k];
      flag[k] = f;
      force_restart[k] = 0;
      if (f) nb[k] = nbnd;
    }
  }
}

// A correction that lost nearly all of its norm to the projection (its
// preconditioned residual lies in the basis, e.g. when H is diagonal in the
// plane waves) is replaced by the residual itself, which is orthogonal to the
// basis: mask[k][r] marks those rows, nrep[k] = nnc[k] where k has one (the
// rows then projected again), else 0.
__global__ __launch_bounds__(64) void dav_residual_mask_kernel(int nbnd, const double* __restrict__ n0,
                                                               const double* __restrict__ n1, const int* nnc,
                                                               int* mask, int* nrep) {
  const int k = blockIdx.x, r = threadIdx.x;
  bool m = false;
  if (r < nbnd) {
    const long o = (long)k * nbnd + r;
    m = r < nnc[k] && !(n1[o] > 1e-8 * n0[o]);
    mask[o] = m;
  }
  const unsigned long long b = __ballot(m);
  if (r == 0) nrep[k] = b ? nnc[k] : 0;
}

// A block whose overlap is numerically singular drops its new rows; the k
// restarts at its next iteration.
__global__ void dav_chol_fail_kernel(int nk, const int* info, int* nnc, int* force_restart) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < nk && info[k] && nnc[k] > 0) {
    nnc[k] = 0;
    force_restart[k] = 1;
  }
}

// The new rows join the basis: nbo = old size (where they start), nb grows by
// nnc; the Rayleigh-Ritz step works on nr = nb rows and forms ny = nbnd Ritz
// vectors for the active k (0 for the frozen ones); hrows counts the rows H
// was applied to.
__global__ void dav_advance_kernel(int nk, int nbnd, int* nb, int* nbo, const int* nnc, const int* active, int* nr,
                                   int* ny, long long* hrows) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  const int b = nb[k], t = b + nnc[k];
  nbo[k] = b;
  nb[k] = t;
  nr[k] = active[k] ? t : 0;
  ny[k] = active[k] ? nbnd : 0;
  hrows[k] += nnc[k];
}

}  // namespace

pw_status davidson_run(pw_ctx* c, pw_prec prec, int nbnd, cd* psi, double* eig, double tol_ry, int max_iter,
                       int32_t* iters_out, int32_t* conv_out) {
  hipStream_t st = c->stream;
  const int nk = c->nk, npwx = c->npwx;
  const int nbmax = std::min<int>((int)c->dav_basis_factor * nbnd, 64);
  const double tol = 0.5 * tol_ry;  // Ha
  const double rtol64 = 1e-5;
  const double tol32 = std::max(tol, 2e-6), rtol32 = 1e-7 * (double)c->mixed_switch_rtol_e7;
  const int nconv = c->dav_nconv > 0 && c->dav_nconv < nbnd ? (int)c->dav_nconv : nbnd;
  const bool gen = c->have_q;  // generalized problem: S != 1
  c->last_iterations = c->last_hpsi_kbands = c->last_graph_replays = 0;
  DevBufs b(c);
  cd *V, *HV, *X, *HX, *T, *Rb, *Hr, *Cr, *Om, *Sm, *Mm;
  cd *SV, *SX;
  double *theta, *rn, *hd, *sd, *nrm0, *nrm1, *th_old;
  int *d_nb, *d_nbo, *d_nnc, *d_nrep, *d_map, *d_flag, *d_active, *d_info, *d_zero, *d_nr, *d_ny, *d_mask;
  int *d_force, *d_iters, *d_nact;
  long long* d_hrows;
  const size_t kb = (size_t)nk * nbmax * npwx, kn = (size_t)nk * nbnd * npwx;
  MKPW_TRY(b.get(kb, &V));
  MKPW_TRY(b.get(kb, &HV));
  MKPW_TRY(b.get(kn, &X));
  MKPW_TRY(b.get(kn, &HX));
  if (gen) {
    MKPW_TRY(b.get(kb, &SV));
    MKPW_TRY(b.get(kn, &SX));
  } else {
    SV = V;  // S = 1: the S-images are the vectors themselves
    SX = X;
  }
  MKPW_TRY(b.get(kn, &T));
  MKPW_TRY(b.get(kn, &Rb));
  MKPW_TRY(b.get((size_t)nk * nbmax * nbmax, &Hr));
  MKPW_TRY(b.get((size_t)nk * nbmax * nbnd, &Cr));
  MKPW_TRY(b.get((size_t)nk * nbmax * nbnd, &Om));
  MKPW_TRY(b.get((size_t)nk * nbnd * nbnd, &Sm));
  MKPW_TRY(b.get((size_t)nk * nbnd * nbnd, &Mm));
  MKPW_TRY(b.get((size_t)nk * nbnd, &theta));
  MKPW_TRY(b.get((size_t)nk * nbnd, &th_old));
  MKPW_TRY(b.get((size_t)nk * nbnd, &rn));
  MKPW_TRY(b.get((size_t)nk * npwx, &hd));
  MKPW_TRY(b.get((size_t)nk * npwx, &sd));
  MKPW_TRY(b.get((size_t)nk * nbnd, &nrm0));
  MKPW_TRY(b.get((size_t)nk * nbnd, &nrm1));
  MKPW_TRY(b.get((size_t)nk, &d_nb));
  MKPW_TRY(b.get((size_t)nk, &d_nbo));
  MKPW_TRY(b.get((size_t)nk, &d_nnc));
  MKPW_TRY(b.get((size_t)nk, &d_nrep));
  MKPW_TRY(b.get((size_t)nk * nbnd, &d_map));
  MKPW_TRY(b.get((size_t)nk, &d_flag));
  MKPW_TRY(b.get((size_t)nk, &d_active));
  MKPW_TRY(b.get((size_t)nk, &d_info));
  MKPW_TRY(b.get((size_t)nk, &d_zero));
  MKPW_TRY(b.get((size_t)nk, &d_nr));
  MKPW_TRY(b.get((size_t)nk, &d_ny));
  MKPW_TRY(b.get((size_t)nk * nbnd, &d_mask));
  MKPW_TRY(b.get((size_t)nk, &d_force));
  MKPW_TRY(b.get((size_t)nk, &d_iters));
  MKPW_TRY(b.get((size_t)nk, &d_hrows));
  MKPW_TRY(b.get((size_t)1, &d_nact));
  cplx<float>*T32 = nullptr, *HT32 = nullptr;
  if (prec == PW_MIXED) {
    MKPW_TRY(b.get(kn, &T32));
    MKPW_TRY(b.get(kn, &HT32));
  }
  const dim3 kgrid((nk + 255) / 256);
  auto fill_i = [&](int* p, long n, int v) {
    hipLaunchKernelGGL(fill_kernel<int>, dim3((unsigned)std::min<long>(1024, (n + 255) / 256)), dim3(256), 0, st, p,
                       n, v);
    return check_launch(c, "fill", st);
  };
  auto fill_c = [&](cd* p, long n) {
    hipLaunchKernelGGL(fill_kernel<cd>, dim3((unsigned)std::min<long>(4096, (n + 255) / 256)), dim3(256), 0, st, p,
                       n, cd{0.0, 0.0});
    return check_launch(c, "fill", st);
  };
  MKPW_TRY(fill_i(d_zero, nk, 0));
  MKPW_TRY(fill_i(d_iters, nk, 0));
  hipLaunchKernelGGL(fill_kernel<long long>, dim3((unsigned)((nk + 255) / 256)), dim3(256), 0, st, d_hrows, (long)nk,
                     0ll);
  MKPW_TRY(check_launch(c, "fill", st));

  // read-back slots for the per-iteration count of active k-points
  HostStage hs(c, st);
  MKPW_TRY(hs.init(0, 2 * sizeof(int) + 256 + sizeof(int) * nk));
  int* slot[2] = {hs.back<int>(0), hs.back<int>(sizeof(int))};
  int* p_nnc = hs.back<int>(256);

  // diagonal of H for the preconditioner
  {
    dim3 grid((npwx + 255) / 256, nk);
    const int np = c->have_proj ? c->nproj : 0;
    hipLaunchKernelGGL(hdiag_kernel, grid, dim3(256), 0, st, c->d_npw, npwx, c->d_kin, c->v0, np,
                       (const cd*)c->d_beta64, (const cd*)c->d_dij64, gen ? (const cd*)c->d_q64 : nullptr, hd, sd);
    MKPW_TRY(check_launch(c, "hdiag", st));
  }

  // Every launch below takes its per-k sizes from device arrays and is sized
  // for their largest possible values (nbnd new rows, nbmax basis rows), so
  // the host never needs them; rows and k-points beyond the per-k counts idle.

  // SV = S V on rows [nb, nb + cnt) (generalized problem only)
  auto apply_s = [&](const int* cnt) -> pw_status {
    if (!gen) return PW_OK;
    VecSel sel;
    sel.nvec = nbnd;
    sel.kstride = (long)nbmax * npwx;
    sel.off = d_nb;
    sel.cnt = cnt;
    return launch_spsi(c, PW_FP64, sel, V, SV, nullptr, 0.0, st);
  };

  // HV = H V on rows [nb, nb + nnc) (FP64, or complex64 through staging rows)
  bool fp64_h = (prec == PW_FP64);
  auto apply_h = [&]() -> pw_status {
    if (fp64_h) {
      VecSel sel;
      sel.nvec = nbnd;
      sel.kstride = (long)nbmax * npwx;
      sel.off = d_nb;
      sel.cnt = d_nnc;
      return launch_hpsi(c, PW_FP64, sel, V, HV, st);
    }
    MKPW_TRY(launch_to_c64(c, V, (long)nbmax * npwx, d_nb, T32, (long)nbnd * npwx, nullptr, d_nnc, nbnd, st));
    VecSel sel;
    sel.nvec = nbnd;
    sel.kstride = (long)nbnd * npwx;
    sel.cnt = d_nnc;
    MKPW_TRY(launch_hpsi(c, PW_MIXED, sel, T32, HT32, st));
    return launch_to_c128(c, HT32, (long)nbnd * npwx, nullptr, HV, (long)nbmax * npwx, d_nb, d_nnc, nbnd, st);
  };

  // rows [nb, nb + cnt): remove the components along rows [0, nb) in the S
  // inner product (twice) and normalise; the norms before (nrm0) and after
  // (nrm1) the projection are kept.  SV follows every row operation on V.
  cd* SV2 = gen ? SV : nullptr;
  auto project = [&](const int* cnt) -> pw_status {
    dim3 grid(nbnd, nk);
    hipLaunchKernelGGL(normalize_rows_kernel, grid, dim3(256), 0, st, V, SV2, (long)nbmax * npwx, d_nb, cnt, npwx,
                       nrm0, nbnd, 0);
    MKPW_TRY(check_launch(c, "norm", st));
    for (int pass = 0; pass < 2; ++pass) {
      GramArgs g;
      g.A = SV; g.a_kstride = (long)nbmax * npwx; g.a_off = d_zero; g.a_cnt = d_nb;
      g.B = V; g.b_kstride = (long)nbmax * npwx; g.b_off = d_nb; g.b_cnt = cnt;
      g.ld = npwx; g.npw = c->d_npw;
      g.C = Om; g.c_kstride = (long)nbmax * nbnd; g.ldc = nbnd;
      MKPW_TRY(launch_gram(c, g, nbmax, nbnd, st));
      CombArgs m;
      m.X = V; m.x_kstride = (long)nbmax * npwx; m.x_off = d_zero; m.x_cnt = d_nb;
      m.Y = V; m.y_kstride = (long)nbmax * npwx; m.y_off = d_nb; m.y_cnt = cnt;
      m.ld = npwx; m.Cm = Om; m.c_kstride = (long)nbmax * nbnd; m.ldc = nbnd;
      m.alpha = -1.0; m.accumulate = 1;
      MKPW_TRY(launch_combine(c, m, nbmax, st));
      if (gen) {
        m.X = SV;
        m.Y = SV;
        MKPW_TRY(launch_combine(c, m, nbmax, st));
      }
    }
    hipLaunchKernelGGL(normalize_rows_kernel, grid, dim3(256), 0, st, V, SV2, (long)nbmax * npwx, d_nb, cnt, npwx,
                       nrm1, nbnd, 1);
    return check_launch(c, "normalize", st);
  };

  // Cholesky-orthonormalise rows [nb, nb + nnc) among themselves in the S inner
  // product (twice); a k whose block is numerically dependent drops its new rows
  // and restarts next time
  auto cholqr = [&]() -> pw_status {
    for (int pass = 0; pass < 2; ++pass) {
      GramArgs g;
      g.A = V; g.a_kstride = (long)nbmax * npwx; g.a_off = d_nb; g.a_cnt = d_nnc;
      g.B = SV; g.b_kstride = (long)nbmax * npwx; g.b_off = d_nb; g.b_cnt = d_nnc;
      g.ld = npwx; g.npw = c->d_npw;
      g.C = Sm; g.c_kstride = (long)nbnd * nbnd; g.ldc = nbnd;
      MKPW_TRY(launch_gram(c, g, nbnd, nbnd, st));
      MKPW_TRY(launch_chol_inv(c, Sm, (long)nbnd * nbnd, nbnd, d_nnc, Mm, (long)nbnd * nbnd, nbnd, d_info, st));
      hipLaunchKernelGGL(dav_chol_fail_kernel, kgrid, dim3(256), 0, st, nk, d_info, d_nnc, d_force);
      MKPW_TRY(check_launch(c, "chol_fail", st));
      MKPW_TRY(launch_trmm(c, V, (long)nbmax * npwx, d_nb, d_nnc, Mm, (long)nbnd * nbnd, nbnd, st));
      if (gen) MKPW_TRY(launch_trmm(c, SV, (long)nbmax * npwx, d_nb, d_nnc, Mm, (long)nbnd * nbnd, nbnd, st));
    }
    return PW_OK;
  };

  // new basis rows from the corrections, with the residual in place of a
  // correction that the projection annihilates
  auto orthonormalize = [&](bool allow_residual) -> pw_status {
    MKPW_TRY(project(d_nnc));
    if (allow_residual) {
      hipLaunchKernelGGL(dav_residual_mask_kernel, dim3(nk), dim3(64), 0, st, nbnd, nrm0, nrm1, d_nnc, d_mask, d_nrep);
      MKPW_TRY(check_launch(c, "residual_mask", st));
      dim3 grid((npwx + 255) / 256, nk, nbnd);
      hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(256), 0, st, Rb, nbnd, V, nbmax, d_nb, d_nrep, d_map, npwx,
                         d_mask);
      MKPW_TRY(check_launch(c, "gather_r", st));
      MKPW_TRY(apply_s(d_nrep));
      MKPW_TRY(project(d_nrep));
    }
    return cholqr();
  };

  // the new rows join the basis; extend H~ by rows [0, nb) x cols [nbo, nb) =
  // V^H HV_new (and the mirrored entries); diagonalise; X = V C, HX = HV C (and
  // S X) for the active k-points (the others keep their converged Ritz pairs)
  auto extend_and_ritz = [&]() -> pw_status {
    hipLaunchKernelGGL(dav_advance_kernel, kgrid, dim3(256), 0, st, nk, nbnd, d_nb, d_nbo, d_nnc, d_active, d_nr, d_ny,
                       d_hrows);
    MKPW_TRY(check_launch(c, "advance", st));
    GramArgs g;
    g.A = V; g.a_kstride = (long)nbmax * npwx; g.a_off = d_zero; g.a_cnt = d_nb;
    g.B = HV; g.b_kstride = (long)nbmax * npwx; g.b_off = d_nbo; g.b_cnt = d_nnc;
    g.ld = npwx; g.npw = c->d_npw;
    g.C = Hr; g.c_kstride = (long)nbmax * nbmax; g.ldc = nbmax; g.c_roff = d_zero; g.c_coff = d_nbo;
    g.mirror = 1;
    MKPW_TRY(launch_gram(c, g, nbmax, nbnd, st));
    MKPW_TRY(launch_heev(c, Hr, (long)nbmax * nbmax, nbmax, d_nr, nbmax, nbnd, theta, Cr, (long)nbmax * nbnd, nbnd, st));
    for (int which = 0; which < 2; ++which) {
      CombArgs m;
      m.X = which ? HV : V; m.x_kstride = (long)nbmax * npwx; m.x_cnt = d_nr;
      m.Y = which ? HX : X; m.y_kstride = (long)nbnd * npwx; m.y_n = nbnd;
      m.y_cnt = d_ny;
      m.ld = npwx; m.Cm = Cr; m.c_kstride = (long)nbmax * nbnd; m.ldc = nbnd;
      MKPW_TRY(launch_combine(c, m, nbmax, st));
    }
    if (gen) {
      // S X afresh rather than SV C: the S-images carried along with the basis
      // drift by rounding over the row updates, and the residuals, the next
      // restart and the final S-orthonormality all read SX
      VecSel sel;
      sel.nvec = nbnd;
      sel.kstride = (long)nbnd * npwx;
      sel.cnt = d_ny;
      MKPW_TRY(launch_spsi(c, PW_FP64, sel, X, SX, nullptr, 0.0, st));
    }
    return PW_OK;
  };

  // one iteration: residuals, the device-side decisions, restarts, corrections,
  // orthonormalisation, H on the new rows, Rayleigh-Ritz
  auto iteration = [&](double etol, double rtol) -> pw_status {
    MKPW_TRY(fill_i(d_nact, 1, 0));
    {
      dim3 grid(nbnd, nk);
      hipLaunchKernelGGL(resid_kernel, grid, dim3(256), 0, st, SX, HX, theta, d_active, hd, sd, c->d_npw, npwx, nbnd,
                         T, Rb, rn);
      MKPW_TRY(check_launch(c, "resid", st));
    }
    hipLaunchKernelGGL(dav_decide_kernel, dim3(nk), dim3(64), 0, st, nbnd, nconv, nbmax, etol, rtol, theta, rn, th_old,
                       d_active, d_nb, d_nnc, d_flag, d_map, d_force, d_iters, d_nact);
    MKPW_TRY(check_launch(c, "decide", st));
    {
      dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
      hipLaunchKernelGGL(restart_kernel, grid, dim3(256), 0, st, d_flag, X, HX, gen ? SX : nullptr, V, HV, SV, nbnd,
                         nbmax, npwx, Hr, theta);
      MKPW_TRY(check_launch(c, "restart", st));
    }
    {
      dim3 grid((npwx + 255) / 256, nk, nbnd);
      hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(256), 0, st, T, nbnd, V, nbmax, d_nb, d_nnc, d_map, npwx,
                         (const int*)nullptr);
      MKPW_TRY(check_launch(c, "gather", st));
    }
    MKPW_TRY(apply_s(d_nnc));
    MKPW_TRY(orthonormalize(true));
    MKPW_TRY(apply_h());
    return extend_and_ritz();
  };

  // (re)start every k from the nbnd rows in V[0:nbnd] (and SV when `have_sv`):
  // orthonormalise them unless they already are, H on them, Rayleigh-Ritz
  auto start = [&](bool orthonormal) -> pw_status {
    hipLaunchKernelGGL(dav_reset_kernel, kgrid, dim3(256), 0, st, nk, nbnd, d_nb, d_nnc, d_active, d_force, th_old);
    MKPW_TRY(check_launch(c, "reset", st));
    if (!orthonormal) {
      MKPW_TRY(apply_s(d_nnc));
      MKPW_TRY(orthonormalize(false));
      MKPW_HIP(c, hipMemcpyAsync(p_nnc, d_nnc, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
      MKPW_HIP(c, hipStreamSynchronize(st));
      for (int k = 0; k < nk; ++k)
        if (p_nnc[k] == 0)
          return set_err(c, PW_EINVAL,
                         std::string("starting vectors are linearly dependent") +
                             (gen ? " (or S is not positive definite)" : "") + " at k " + std::to_string(k));
    }
    MKPW_TRY(apply_h());
    MKPW_TRY(fill_c(Hr, (long)nk * nbmax * nbmax));
    return extend_and_ritz();
  };

  // ---- start: V[0:nbnd] = psi
  {
    dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
    hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, psi, nbnd, V, nbmax, nbnd, npwx);
    MKPW_TRY(check_launch(c, "copy", st));
  }
  MKPW_TRY(start(false));

  // ---- iterations.  The host learns whether any k is still active one
  // iteration late (the count is copied to page-locked memory behind each
  // iteration and read once the next one is queued), so the device never
  // waits for it; an iteration queued after every k has converged changes
  // nothing.  From the second iteration of a phase on, the iteration runs as
  // a captured graph, replayed.
  hipEvent_t ev[2] = {nullptr, nullptr};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  struct Cleanup {
    hipEvent_t* e;
    hipGraph_t* g;
    hipGraphExec_t* x;
    ~Cleanup() {
      for (int i = 0; i < 2; ++i)
        if (e[i]) (void)hipEventDestroy(e[i]);
      if (*x) (void)hipGraphExecDestroy(*x);
      if (*g) (void)hipGraphDestroy(*g);
    }
  } cleanup{ev, &graph, &exec};
  for (int i = 0; i < 2; ++i) MKPW_HIP(c, hipEventCreateWithFlags(&ev[i], hipEventDisableTiming));
  bool use_graph = c->solver_graph && !c->trace;
  auto drop_graph = [&]() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };
  auto run_iteration = [&](int in_phase, double etol, double rtol) -> pw_status {
    if (use_graph && in_phase >= 2) {
      if (!exec) {
        bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
          pw_status s = iteration(etol, rtol);
          hipGraph_t g = nullptr;
          const bool ended = hipStreamEndCapture(st, &g) == hipSuccess;
          if (s != PW_OK) {
            if (g) (void)hipGraphDestroy(g);
            return s;
          }
          ok = ended && g && hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
          graph = g;
        }
        if (!ok) {  // run this and every later iteration launch by launch
          (void)hipGetLastError();
          drop_graph();
          use_graph = false;
          return iteration(etol, rtol);
        }
      }
      MKPW_HIP(c, hipGraphLaunch(exec, st));
      ++c->last_graph_replays;
      return PW_OK;
    }
    return iteration(etol, rtol);
  };

  bool refine = false;  // mixed precision: FP64 phase started
  bool all_done = false;
  int phase_first = 1;  // first iteration of the current phase
  int it = 0;
  for (it = 1;; ++it) {
    if (it <= max_iter) {
      const double etol = fp64_h ? tol : tol32, rtol = fp64_h ? rtol64 : rtol32;
      MKPW_TRY(run_iteration(it - phase_first + 1, etol, rtol));
      MKPW_HIP(c, hipMemcpyAsync(slot[it & 1], d_nact, sizeof(int), hipMemcpyDeviceToHost, st));
      MKPW_HIP(c, hipEventRecord(ev[it & 1], st));
    }
    if (it > phase_first) {
      MKPW_HIP(c, hipEventSynchronize(ev[(it - 1) & 1]));
      if (*slot[(it - 1) & 1] == 0) {
        if (prec == PW_MIXED && !refine && c->mixed_refine) {
          // FP64 refinement: restart every k from its Ritz vectors with H in FP64
          refine = true;
          fp64_h = true;
          drop_graph();
          dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
          hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, X, nbnd, V, nbmax, nbnd, npwx);
          MKPW_TRY(check_launch(c, "copy", st));
          if (gen) {
            hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, SX, nbnd, SV, nbmax, nbnd, npwx);
            MKPW_TRY(check_launch(c, "copy", st));
          }
          MKPW_TRY(start(true));
          phase_first = it + 1;
          continue;
        }
        all_done = true;
        break;
      }
    }
    if (it > max_iter) break;
  }
  c->last_iterations = std::min(it, max_iter);

  // results: Ritz vectors and values, per-k counts
  {
    dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
    hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, X, nbnd, psi, nbnd, nbnd, npwx);
    MKPW_TRY(check_launch(c, "copy", st));
  }
  std::vector<int> iters(nk), active(nk);
  std::vector<long long> hrows(nk);
  MKPW_HIP(c, hipMemcpyAsync(eig, theta, sizeof(double) * (size_t)nk * nbnd, hipMemcpyDeviceToHost, st));
  MKPW_HIP(c, hipMemcpyAsync(iters.data(), d_iters, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
  MKPW_HIP(c, hipMemcpyAsync(active.data(), d_active, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
  MKPW_HIP(c, hipMemcpyAsync(hrows.data(), d_hrows, sizeof(long long) * nk, hipMemcpyDeviceToHost, st));
  MKPW_HIP(c, hipStreamSynchronize(st));
  bool all_conv = true;
  for (int k = 0; k < nk; ++k) {
    if (iters_out) iters_out[k] = iters[k];
    if (conv_out) conv_out[k] = active[k] ? 0 : 1;
    if (active[k]) all_conv = false;
    c->last_hpsi_kbands += hrows[k];
  }
  if (!all_done || !all_conv) return set_err(c, PW_ENOCONV, "Davidson: some k-points did not converge");
  return PW_OK;
}

}  // namespace mkpw

extern "C" pw_status pw_davidson(pw_ctx* c, pw_prec prec, int nbnd, void* psi, double* eig, double tol_ry,
                                 int max_iter, int32_t* iters, int32_t* converged) {
  using namespace mkpw;
  if (!c) return PW_EINVAL;
  if (c->host_only) return set_err(c, PW_ESTATE, "host-only context runs no device work");
  if (!c->have_k || !c->have_v) return set_err(c, PW_ESTATE, "set k-points and potential before davidson");
  if (prec != PW_FP64 && prec != PW_MIXED) return set_err(c, PW_EINVAL, "unknown precision");
  if (!psi || !eig) return set_err(c, PW_EINVAL, "null psi or eig");
  if (nbnd < 1 || nbnd > 32) return set_err(c, PW_EINVAL, "nbnd must be in [1, 32]");
  int npwmin = *std::min_element(c->npw.begin(), c->npw.end());
  if (2 * nbnd > npwmin) return set_err(c, PW_EINVAL, "nbnd exceeds half the smallest basis");
  if (!(tol_ry > 0.0)) return set_err(c, PW_EINVAL, "tol_ry must be positive");
  if (max_iter < 1) return set_err(c, PW_EINVAL, "max_iter must be >= 1");
  (void)hipSetDevice(c->device);
  return davidson_run(c, prec, nbnd, (cplx<double>*)psi, eig, tol_ry, max_iter, iters, converged);
}
