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

}  // namespace

pw_status davidson_run(pw_ctx* c, pw_prec prec, int nbnd, cd* psi, double* eig, double tol_ry, int max_iter,
                       int32_t* iters_out, int32_t* conv_out) {
  hipStream_t st = c->stream;
  const int nk = c->nk, npwx = c->npwx;
  const int nbmax = std::min<int>((int)c->dav_basis_factor * nbnd, 64);
  const double tol = 0.5 * tol_ry;  // Ha
  const double rtol64 = 1e-5;
  const double tol32 = std::max(tol, 2e-6), rtol32 = 2e-4;
  const bool gen = c->have_q;  // generalized problem: S != 1
  DevBufs b(c);
  cd *V, *HV, *X, *HX, *T, *Rb, *Hr, *Cr, *Om, *Sm, *Mm;
  cd *SV, *SX;
  double *theta, *rn, *hd, *sd, *nrm0, *nrm1;
  int *d_nb, *d_nnc, *d_map, *d_flag, *d_active, *d_info, *d_zero, *d_nr, *d_ny, *d_ntot, *d_mask;
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
  MKPW_TRY(b.get((size_t)nk * nbnd, &rn));
  MKPW_TRY(b.get((size_t)nk * npwx, &hd));
  MKPW_TRY(b.get((size_t)nk * npwx, &sd));
  MKPW_TRY(b.get((size_t)nk * nbnd, &nrm0));
  MKPW_TRY(b.get((size_t)nk * nbnd, &nrm1));
  MKPW_TRY(b.get((size_t)nk, &d_nb));
  MKPW_TRY(b.get((size_t)nk, &d_nnc));
  MKPW_TRY(b.get((size_t)nk * nbnd, &d_map));
  MKPW_TRY(b.get((size_t)nk, &d_flag));
  MKPW_TRY(b.get((size_t)nk, &d_active));
  MKPW_TRY(b.get((size_t)nk, &d_info));
  MKPW_TRY(b.get((size_t)nk, &d_zero));
  MKPW_TRY(b.get((size_t)nk, &d_nr));
  MKPW_TRY(b.get((size_t)nk, &d_ny));
  MKPW_TRY(b.get((size_t)nk, &d_ntot));
  MKPW_TRY(b.get((size_t)nk * nbnd, &d_mask));
  cplx<float>*T32 = nullptr, *HT32 = nullptr;
  if (prec == PW_MIXED) {
    MKPW_TRY(b.get(kn, &T32));
    MKPW_TRY(b.get(kn, &HT32));
  }
  MKPW_HIP(c, hipMemsetAsync(d_zero, 0, sizeof(int) * nk, st));

  // host mirrors
  std::vector<int> nb(nk, 0), nnc(nk, nbnd), map((size_t)nk * nbnd), flag(nk, 0), active(nk, 1), info(nk, 0);
  std::vector<double> th((size_t)nk * nbnd), th_old((size_t)nk * nbnd, std::numeric_limits<double>::infinity()),
      rnh((size_t)nk * nbnd);
  std::vector<int> iters(nk, 0);
  std::vector<int> force_restart(nk, 0);
  // uploads go through page-locked snapshots, so the host arrays may change
  // right after a call; the per-k read-backs land in page-locked memory too
  // (between two synchronisations an iteration uploads at most ten (nk) arrays
  // and two (nk, nbnd) ones)
  const size_t nkb = (size_t)nk * nbnd;
  HostStage hs(c, st);
  MKPW_TRY(hs.init(sizeof(int) * (16 * (size_t)nk + 2 * nkb) + 256 * 24, sizeof(double) * 4 * nkb + sizeof(int) * nk));
  double* p_th = hs.back<double>(0);
  double* p_rn = p_th + nkb;
  double* p_n0 = p_rn + nkb;
  double* p_n1 = p_n0 + nkb;
  int* p_info = reinterpret_cast<int*>(p_n1 + nkb);
  auto h2d = [&](int* d, const std::vector<int>& h) { return hs.up(d, h.data(), h.size()); };
  auto sync = [&]() { return hs.sync(); };

  // diagonal of H for the preconditioner
  {
    dim3 grid((npwx + 255) / 256, nk);
    const int np = c->have_proj ? c->nproj : 0;
    hipLaunchKernelGGL(hdiag_kernel, grid, dim3(256), 0, st, c->d_npw, npwx, c->d_kin, c->v0, np,
                       (const cd*)c->d_beta64, (const cd*)c->d_dij64, gen ? (const cd*)c->d_q64 : nullptr, hd, sd);
    MKPW_TRY(check_launch(c, "hdiag", st));
  }

  // SV = S V on rows [nb, nb + nnc) (generalized problem only)
  auto apply_s = [&](int nvec_max) -> pw_status {
    if (!gen || nvec_max <= 0) return PW_OK;
    VecSel sel;
    sel.nvec = nvec_max;
    sel.kstride = (long)nbmax * npwx;
    sel.off = d_nb;
    sel.cnt = d_nnc;
    return launch_spsi(c, PW_FP64, sel, V, SV, nullptr, 0.0, st);
  };

  // apply H to rows [nb, nb + nnc) of V into HV (FP64 or complex64 staging)
  bool fp64_h = (prec == PW_FP64);
  auto apply_h = [&](int nvec_max) -> pw_status {
    if (nvec_max <= 0) return PW_OK;
    if (fp64_h) {
      VecSel sel;
      sel.nvec = nvec_max;
      sel.kstride = (long)nbmax * npwx;
      sel.off = d_nb;
      sel.cnt = d_nnc;
      MKPW_TRY(launch_hpsi(c, PW_FP64, sel, V, HV, st));
      return PW_OK;
    }
    MKPW_TRY(launch_to_c64(c, V, (long)nbmax * npwx, d_nb, T32, (long)nbnd * npwx, nullptr, d_nnc, nvec_max, st));
    VecSel sel;
    sel.nvec = nvec_max;
    sel.kstride = (long)nbnd * npwx;
    sel.cnt = d_nnc;
    MKPW_TRY(launch_hpsi(c, PW_MIXED, sel, T32, HT32, st));
    MKPW_TRY(launch_to_c128(c, HT32, (long)nbnd * npwx, nullptr, HV, (long)nbmax * npwx, d_nb, d_nnc, nvec_max, st));
    return PW_OK;
  };

  // rows [nb, nb + nnc): remove the components along rows [0, nb) in the S
  // inner product (twice) and normalise; the norms before (nrm0) and after
  // (nrm1) the projection are kept.  SV follows every row operation on V.
  cd* SV2 = gen ? SV : nullptr;
  auto project = [&](int nb_max, int nnc_max) -> pw_status {
    if (nnc_max <= 0) return PW_OK;
    dim3 grid(nnc_max, nk);
    hipLaunchKernelGGL(normalize_rows_kernel, grid, dim3(256), 0, st, V, SV2, (long)nbmax * npwx, d_nb, d_nnc, npwx,
                       nrm0, nbnd, 0);
    MKPW_TRY(check_launch(c, "norm", st));
    for (int pass = 0; pass < 2 && nb_max > 0; ++pass) {
      GramArgs g;
      g.A = SV; g.a_kstride = (long)nbmax * npwx; g.a_off = d_zero; g.a_cnt = d_nb;
      g.B = V; g.b_kstride = (long)nbmax * npwx; g.b_off = d_nb; g.b_cnt = d_nnc;
      g.ld = npwx; g.npw = c->d_npw;
      g.C = Om; g.c_kstride = (long)nbmax * nbnd; g.ldc = nbnd;
      MKPW_TRY(launch_gram(c, g, nb_max, nnc_max, st));
      CombArgs m;
      m.X = V; m.x_kstride = (long)nbmax * npwx; m.x_off = d_zero; m.x_cnt = d_nb;
      m.Y = V; m.y_kstride = (long)nbmax * npwx; m.y_off = d_nb; m.y_cnt = d_nnc;
      m.ld = npwx; m.Cm = Om; m.c_kstride = (long)nbmax * nbnd; m.ldc = nbnd;
      m.alpha = -1.0; m.accumulate = 1;
      MKPW_TRY(launch_combine(c, m, nb_max, st));
      if (gen) {
        m.X = SV;
        m.Y = SV;
        MKPW_TRY(launch_combine(c, m, nb_max, st));
      }
    }
    hipLaunchKernelGGL(normalize_rows_kernel, grid, dim3(256), 0, st, V, SV2, (long)nbmax * npwx, d_nb, d_nnc, npwx,
                       nrm1, nbnd, 1);
    return check_launch(c, "normalize", st);
  };

  // Cholesky-orthonormalise rows [nb, nb + nnc) among themselves in the S inner
  // product (twice); a k whose block is numerically dependent drops its new rows
  // and restarts next time
  auto cholqr = [&](int nnc_max) -> pw_status {
    if (nnc_max <= 0) return PW_OK;
    for (int pass = 0; pass < 2; ++pass) {
      GramArgs g;
      g.A = V; g.a_kstride = (long)nbmax * npwx; g.a_off = d_nb; g.a_cnt = d_nnc;
      g.B = SV; g.b_kstride = (long)nbmax * npwx; g.b_off = d_nb; g.b_cnt = d_nnc;
      g.ld = npwx; g.npw = c->d_npw;
      g.C = Sm; g.c_kstride = (long)nbnd * nbnd; g.ldc = nbnd;
      MKPW_TRY(launch_gram(c, g, nnc_max, nnc_max, st));
      MKPW_TRY(launch_chol_inv(c, Sm, (long)nbnd * nbnd, nbnd, d_nnc, Mm, (long)nbnd * nbnd, nbnd, d_info, st));
      MKPW_TRY(launch_trmm(c, V, (long)nbmax * npwx, d_nb, d_nnc, Mm, (long)nbnd * nbnd, nbnd, st));
      if (gen) MKPW_TRY(launch_trmm(c, SV, (long)nbmax * npwx, d_nb, d_nnc, Mm, (long)nbnd * nbnd, nbnd, st));
      MKPW_HIP(c, hipMemcpyAsync(p_info, d_info, sizeof(int) * nk, hipMemcpyDeviceToHost, st));
      MKPW_HIP(c, sync());
      std::memcpy(info.data(), p_info, sizeof(int) * nk);
      bool changed = false;
      for (int k = 0; k < nk; ++k)
        if (info[k] && nnc[k] > 0) {
          nnc[k] = 0;
          force_restart[k] = 1;
          changed = true;
        }
      if (changed) MKPW_HIP(c, h2d(d_nnc, nnc));
    }
    return PW_OK;
  };

  // new basis rows from the corrections; a correction that loses nearly all of
  // its norm to the projection (the preconditioned residual lies in the basis,
  // e.g. when H is diagonal in the plane waves) is replaced by the residual
  // itself, which is orthogonal to the basis by construction
  std::vector<double> n0h((size_t)nk * nbnd), n1h((size_t)nk * nbnd);
  std::vector<int> mask((size_t)nk * nbnd);
  auto orthonormalize = [&](int nb_max, int nnc_max, bool allow_residual) -> pw_status {
    if (nnc_max <= 0) return PW_OK;
    MKPW_TRY(project(nb_max, nnc_max));
    if (allow_residual) {
      MKPW_HIP(c, hipMemcpyAsync(p_n0, nrm0, sizeof(double) * nkb, hipMemcpyDeviceToHost, st));
      MKPW_HIP(c, hipMemcpyAsync(p_n1, nrm1, sizeof(double) * nkb, hipMemcpyDeviceToHost, st));
      MKPW_HIP(c, sync());
      std::memcpy(n0h.data(), p_n0, sizeof(double) * nkb);
      std::memcpy(n1h.data(), p_n1, sizeof(double) * nkb);
      bool any = false;
      for (int k = 0; k < nk; ++k)
        for (int r = 0; r < nbnd; ++r) {
          const size_t o = (size_t)k * nbnd + r;
          mask[o] = (r < nnc[k]) && !(n1h[o] > 1e-8 * n0h[o]);
          any = any || mask[o];
        }
      if (any) {
        MKPW_HIP(c, h2d(d_mask, mask));
        dim3 grid((npwx + 255) / 256, nk, nnc_max);
        hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(256), 0, st, Rb, nbnd, V, nbmax, d_nb, d_nnc, d_map, npwx,
                           d_mask);
        MKPW_TRY(check_launch(c, "gather_r", st));
        MKPW_TRY(apply_s(nnc_max));
        MKPW_TRY(project(nb_max, nnc_max));
      }
    }
    return cholqr(nnc_max);
  };

  // extend H~: rows [0, nb + nnc) x cols [nb, nb + nnc) = V^H HV_new (+ mirror)
  auto extend_h = [&](int ntot_max, int nnc_max) -> pw_status {
    std::vector<int> ntot(nk);
    for (int k = 0; k < nk; ++k) ntot[k] = nb[k] + nnc[k];
    MKPW_HIP(c, h2d(d_ntot, ntot));
    GramArgs g;
    g.A = V; g.a_kstride = (long)nbmax * npwx; g.a_off = d_zero; g.a_cnt = d_ntot;
    g.B = HV; g.b_kstride = (long)nbmax * npwx; g.b_off = d_nb; g.b_cnt = d_nnc;
    g.ld = npwx; g.npw = c->d_npw;
    g.C = Hr; g.c_kstride = (long)nbmax * nbmax; g.ldc = nbmax; g.c_roff = d_zero; g.c_coff = d_nb;
    g.mirror = 1;
    MKPW_TRY(launch_gram(c, g, ntot_max, nnc_max, st));
    return PW_OK;
  };

  std::vector<int> nr(nk), ny(nk);
  auto ritz = [&](int nb_max) -> pw_status {
    // nb := nb + nnc has been applied; diagonalise and form X, HX for the
    // active k-points (the others keep their converged Ritz pairs)
    for (int k = 0; k < nk; ++k) {
      nr[k] = active[k] ? nb[k] : 0;
      ny[k] = active[k] ? nbnd : 0;
    }
    MKPW_HIP(c, h2d(d_nb, nb));
    MKPW_HIP(c, h2d(d_nr, nr));
    MKPW_HIP(c, h2d(d_ny, ny));
    MKPW_TRY(launch_heev(c, Hr, (long)nbmax * nbmax, nbmax, d_nr, nb_max, nbnd, theta, Cr, (long)nbmax * nbnd, nbnd, st));
    for (int which = 0; which < 2; ++which) {
      CombArgs m;
      m.X = which ? HV : V; m.x_kstride = (long)nbmax * npwx; m.x_cnt = d_nr;
      m.Y = which ? HX : X; m.y_kstride = (long)nbnd * npwx; m.y_n = nbnd;
      m.y_cnt = d_ny;
      m.ld = npwx; m.Cm = Cr; m.c_kstride = (long)nbmax * nbnd; m.ldc = nbnd;
      MKPW_TRY(launch_combine(c, m, nb_max, st));
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

  // ---- start: V[0:nbnd] = psi, orthonormalise, H V, H~, Ritz pairs
  {
    dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
    hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, psi, nbnd, V, nbmax, nbnd, npwx);
    MKPW_TRY(check_launch(c, "copy", st));
    std::fill(nb.begin(), nb.end(), 0);
    std::fill(nnc.begin(), nnc.end(), nbnd);
    MKPW_HIP(c, h2d(d_nb, nb));
    MKPW_HIP(c, h2d(d_nnc, nnc));
    MKPW_TRY(apply_s(nbnd));
    MKPW_TRY(orthonormalize(0, nbnd, false));
    for (int k = 0; k < nk; ++k)
      if (nnc[k] == 0) return set_err(c, PW_EINVAL,
                       std::string("starting vectors are linearly dependent") +
                           (gen ? " (or S is not positive definite)" : "") + " at k " + std::to_string(k));
    MKPW_TRY(apply_h(nbnd));
    MKPW_HIP(c, hipMemsetAsync(Hr, 0, sizeof(cd) * (size_t)nk * nbmax * nbmax, st));
    MKPW_TRY(extend_h(nbnd, nbnd));
    for (int k = 0; k < nk; ++k) nb[k] = nbnd;
    MKPW_TRY(ritz(nbnd));
  }

  bool refine = false;  // mixed precision: FP64 phase started
  int it = 0;
  bool all_done = false;
  for (it = 1; it <= max_iter; ++it) {
    // residuals of the current Ritz pairs
    MKPW_HIP(c, h2d(d_active, active));
    {
      dim3 grid(nbnd, nk);
      hipLaunchKernelGGL(resid_kernel, grid, dim3(256), 0, st, SX, HX, theta, d_active, hd, sd, c->d_npw, npwx, nbnd,
                         T, Rb, rn);
      MKPW_TRY(check_launch(c, "resid", st));
    }
    MKPW_HIP(c, hipMemcpyAsync(p_th, theta, sizeof(double) * nkb, hipMemcpyDeviceToHost, st));
    MKPW_HIP(c, hipMemcpyAsync(p_rn, rn, sizeof(double) * nkb, hipMemcpyDeviceToHost, st));
    MKPW_HIP(c, sync());
    std::memcpy(th.data(), p_th, sizeof(double) * nkb);
    std::memcpy(rnh.data(), p_rn, sizeof(double) * nkb);
    const double etol = fp64_h ? tol : tol32, rtol = fp64_h ? rtol64 : rtol32;
    int n_active = 0, nnc_max = 0, nb_max = 0;
    for (int k = 0; k < nk; ++k) {
      if (!active[k]) {
        nnc[k] = 0;
        flag[k] = 0;
        continue;
      }
      iters[k] = it;
      int cnt = 0;
      for (int j = 0; j < nbnd; ++j) {
        const size_t o = (size_t)k * nbnd + j;
        bool ok = std::fabs(th[o] - th_old[o]) < etol && rnh[o] < rtol;
        if (!ok) map[(size_t)k * nbnd + cnt++] = j;
      }
      if (cnt == 0) {
        active[k] = 0;
        nnc[k] = 0;
        flag[k] = 0;
        continue;
      }
      ++n_active;
      nnc[k] = cnt;
      flag[k] = (nb[k] + cnt > nbmax) || force_restart[k];
      force_restart[k] = 0;
      if (flag[k]) nb[k] = nbnd;
      nnc_max = std::max(nnc_max, cnt);
      nb_max = std::max(nb_max, nb[k] + cnt);
    }
    th_old = th;
    if (n_active == 0) {
      if (prec == PW_MIXED && !refine) {
        // FP64 refinement: restart every k from its Ritz vectors with H in FP64
        refine = true;
        fp64_h = true;
        std::fill(active.begin(), active.end(), 1);
        std::fill(th_old.begin(), th_old.end(), std::numeric_limits<double>::infinity());
        dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
        hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, X, nbnd, V, nbmax, nbnd, npwx);
        MKPW_TRY(check_launch(c, "copy", st));
        if (gen) {
          hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, SX, nbnd, SV, nbmax, nbnd, npwx);
          MKPW_TRY(check_launch(c, "copy", st));
        }
        std::fill(nb.begin(), nb.end(), 0);
        std::fill(nnc.begin(), nnc.end(), nbnd);
        MKPW_HIP(c, h2d(d_nb, nb));
        MKPW_HIP(c, h2d(d_nnc, nnc));
        MKPW_TRY(apply_h(nbnd));
        MKPW_HIP(c, hipMemsetAsync(Hr, 0, sizeof(cd) * (size_t)nk * nbmax * nbmax, st));
        MKPW_TRY(extend_h(nbnd, nbnd));
        for (int k = 0; k < nk; ++k) nb[k] = nbnd;
        MKPW_TRY(ritz(nbnd));
        continue;
      }
      all_done = true;
      break;
    }
    MKPW_HIP(c, h2d(d_flag, flag));
    MKPW_HIP(c, h2d(d_map, map));
    MKPW_HIP(c, h2d(d_nnc, nnc));
    {
      dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
      hipLaunchKernelGGL(restart_kernel, grid, dim3(256), 0, st, d_flag, X, HX, gen ? SX : nullptr, V, HV, SV, nbnd,
                         nbmax, npwx, Hr, theta);
      MKPW_TRY(check_launch(c, "restart", st));
    }
    MKPW_HIP(c, h2d(d_nb, nb));
    {
      dim3 grid((npwx + 255) / 256, nk, nnc_max);
      hipLaunchKernelGGL(gather_rows_kernel, grid, dim3(256), 0, st, T, nbnd, V, nbmax, d_nb, d_nnc, d_map, npwx,
                         (const int*)nullptr);
      MKPW_TRY(check_launch(c, "gather", st));
    }
    MKPW_TRY(apply_s(nnc_max));
    int nb_cur_max = 0;
    for (int k = 0; k < nk; ++k) nb_cur_max = std::max(nb_cur_max, nb[k]);
    MKPW_TRY(orthonormalize(nb_cur_max, nnc_max, true));
    MKPW_TRY(apply_h(nnc_max));
    MKPW_TRY(extend_h(nb_max, nnc_max));
    int ntot_max = 0;
    for (int k = 0; k < nk; ++k) {
      nb[k] += nnc[k];
      ntot_max = std::max(ntot_max, nb[k]);
    }
    MKPW_TRY(ritz(ntot_max));
  }

  // results: Ritz vectors and values
  {
    dim3 grid(std::max(1, std::min(64, (nbnd * npwx + 255) / 256)), nk);
    hipLaunchKernelGGL(copy_rows_kernel, grid, dim3(256), 0, st, X, nbnd, psi, nbnd, nbnd, npwx);
    MKPW_TRY(check_launch(c, "copy", st));
  }
  MKPW_HIP(c, hipMemcpyAsync(eig, theta, sizeof(double) * (size_t)nk * nbnd, hipMemcpyDeviceToHost, st));
  MKPW_HIP(c, sync());
  bool all_conv = true;
  for (int k = 0; k < nk; ++k) {
    if (iters_out) iters_out[k] = iters[k];
    if (conv_out) conv_out[k] = active[k] ? 0 : 1;
    if (active[k]) all_conv = false;
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
