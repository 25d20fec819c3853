// Batched overlap operator (Sec. 2.2, Eqs. lambdah, delta_eq and finals):
//   lambda_q = <beta_q|psi>,  delta_p = sum_q q_pq lambda_q,
//   S psi    = psi + sum_p delta_p beta_p
// for every selected (k, band) row at once.  One workgroup per row: the
// waves share the projections (each wave reduces a subset of the nproj
// inner products over the row with DPP sums), then every work-item writes
// its plane waves.  beta of one k is read by all rows of that k, which run
// next to each other in the grid, so it is served from L2; psi is read from
// HBM once and the output written once: the operator is bound by HBM
// bandwidth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.hpp"
#include "wave.hpp"

namespace mkpw {

namespace {

constexpr int kSThreads = 256;
constexpr int kSMaxProj = 32;

template <class T>
__global__ __launch_bounds__(kSThreads) void spsi_kernel(const cplx<T>* psi, cplx<T>* out,
                                                         long kstride, int nvec, const int* __restrict__ off,
                                                         const int* __restrict__ cnt, const int* __restrict__ live,
                                                         const int* __restrict__ npw_k, int npwx, int nproj,
                                                         const cplx<T>* __restrict__ beta,
                                                         const cplx<T>* __restrict__ q,
                                                         const double* __restrict__ scale, double mult) {
  const int k = blockIdx.y, r = blockIdx.x;
  if (r >= (cnt ? cnt[k] : nvec)) return;
  if (live && !live[(long)k * nvec + r]) return;
  const long row = (long)k * kstride + (long)((off ? off[k] : 0) + r) * npwx;
  const cplx<T>* x = psi + row;
  cplx<T>* y = out + row;
  const int npw = npw_k[k];
  const cplx<T>* bk = beta + (long)k * nproj * npwx;
  __shared__ cplx<T> lam[kSMaxProj], dlt[kSMaxProj];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // lambda_p = sum_G conj(beta_p(G)) psi(G)   (Eq. lambdah)
  for (int p = wave; p < nproj; p += kSThreads / 64) {
    const cplx<T>* b = bk + (long)p * npwx;
    T sr = T(0), si = T(0);
    for (int g = lane; g < npw; g += 64) {
      cplx<T> bv = b[g], xv = x[g];
      sr += bv.x * xv.x + bv.y * xv.y;
      si += bv.x * xv.y - bv.y * xv.x;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    if (lane == 0) lam[p] = {sr, si};
  }
  __syncthreads();
  // delta_p = sum_q q_pq lambda_q   (Eq. delta_eq)
  if (threadIdx.x < nproj) {
    const int p = threadIdx.x;
    T dr = T(0), di = T(0);
    for (int s = 0; s < nproj; ++s) {
      cplx<T> qq = q[p * nproj + s], l = lam[s];
      dr += qq.x * l.x - qq.y * l.y;
      di += qq.x * l.y + qq.y * l.x;
    }
    dlt[p] = {dr, di};
  }
  __syncthreads();
  // S psi = psi + sum_p delta_p beta_p   (Eq. finals)
  const T f = scale ? T(mult * scale[(long)k * nvec + r]) : T(1);
  for (int g = threadIdx.x; g < npwx; g += kSThreads) {
    if (g >= npw) {
      if (!scale) y[g] = {T(0), T(0)};
      continue;
    }
    cplx<T> v = x[g];
    for (int p = 0; p < nproj; ++p) {
      cplx<T> bv = bk[(long)p * npwx + g], d = dlt[p];
      v.x += d.x * bv.x - d.y * bv.y;
      v.y += d.x * bv.y + d.y * bv.x;
    }
    if (scale) {
      cplx<T> o = y[g];
      y[g] = {o.x + f * v.x, o.y + f * v.y};
    } else {
      y[g] = v;
    }
  }
}

}  // namespace

pw_status launch_spsi(pw_ctx* c, pw_prec prec, const VecSel& sel, const void* psi, void* out, const double* scale,
                      double mult, hipStream_t st) {
  if (sel.nvec <= 0) return PW_OK;
  const int nproj = c->have_q ? c->nproj : 0;
  if (nproj > kSMaxProj) return set_err(c, PW_EINVAL, "overlap: more than 32 projectors");
  dim3 grid(sel.nvec, c->nk);
  if (prec == PW_FP64) {
    hipLaunchKernelGGL(spsi_kernel<double>, grid, dim3(kSThreads), 0, st, (const cplx<double>*)psi,
                       (cplx<double>*)out, sel.kstride, sel.nvec, sel.off, sel.cnt, sel.live, c->d_npw, c->npwx,
                       nproj, (const cplx<double>*)c->d_beta64, (const cplx<double>*)c->d_q64, scale, mult);
  } else {
    hipLaunchKernelGGL(spsi_kernel<float>, grid, dim3(kSThreads), 0, st, (const cplx<float>*)psi,
                       (cplx<float>*)out, sel.kstride, sel.nvec, sel.off, sel.cnt, sel.live, c->d_npw, c->npwx,
                       nproj, (const cplx<float>*)c->d_beta32, (const cplx<float>*)c->d_q32, scale, mult);
  }
  return check_launch(c, "s_psi", st);
}

}  // namespace mkpw

extern "C" pw_status pw_s_psi(pw_ctx* c, pw_prec prec, int nbnd, const void* psi, void* spsi) {
  using namespace mkpw;
  if (!c) return PW_EINVAL;
  if (c->host_only) return set_err(c, PW_ESTATE, "host-only context runs no device work");
  if (!c->have_k) return set_err(c, PW_ESTATE, "set k-points before s_psi");
  if (prec != PW_FP64 && prec != PW_MIXED) return set_err(c, PW_EINVAL, "unknown precision");
  if (nbnd <= 0 || nbnd > 65535) return set_err(c, PW_EINVAL, "nbnd must be in [1, 65535]");
  if (!psi || !spsi) return set_err(c, PW_EINVAL, "null psi or spsi");
  (void)hipSetDevice(c->device);
  VecSel sel;
  sel.nvec = nbnd;
  sel.kstride = (long)nbnd * c->npwx;
  return launch_spsi(c, prec, sel, psi, spsi, nullptr, 0.0, c->stream);
}
