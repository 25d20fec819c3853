// Batched overlap operator (Sec. 2.2, Eqs. lambdah, delta_eq and finals):
//   lambda_q = <beta_q|psi>,  delta_p = sum_q q_pq lambda_q,
//   S psi    = psi + sum_p delta_p beta_p
// for every selected (k, band) row at once.  One wavefront per row, four
// rows per workgroup: each lane accumulates its plane waves' share of the
// nproj inner products, DPP sums give every lane all of lambda, every lane
// forms delta from q (staged in LDS once per workgroup), and writes its plane
// waves; apart from the q staging no barrier is needed.  Rows are dealt to
// the XCDs so that all rows of a k-point run on one XCD: the projector rows
// of a k are fetched from HBM into one L2 and served from there to all its
// bands.  psi is read from HBM once (its second read, for the output, hits
// L2) and the output written once, so the operator is bound by HBM bandwidth.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "internal.hpp"
#include "wave.hpp"  // dpp<>, wave_sum

namespace mkpw {

namespace {

constexpr int kSThreads = 256;  // four rows per workgroup
constexpr int kSMaxProj = 32;

// NP: nproj rounded up to a multiple of 8 (8 or 32), so that lambda and
// delta live in registers.  NPL > 0: each lane keeps its NPL plane waves
// (g = lane + 64 i) of psi in registers, loaded all at once, so the row is read
// from HBM once with every load in flight together; NPL = 0 (rows longer than
// 16 x 64) loops over the row and reads psi a second time for the output.
template <class T, int NP, int NPL>
__global__ __launch_bounds__(kSThreads) void spsi_kernel(const cplx<T>* psi, cplx<T>* out, long kstride, int nvec,
                                                         const int* __restrict__ off, const int* __restrict__ cnt,
                                                         const int* __restrict__ live, const int* __restrict__ npw_k,
                                                         int npwx, int nproj, const cplx<T>* __restrict__ beta,
                                                         const cplx<T>* __restrict__ q,
                                                         const double* __restrict__ scale, double mult, int per_xcd,
                                                         int ntask) {
  extern __shared__ char smem[];
  auto* qs = reinterpret_cast<cplx<T>*>(smem);  // q, nproj x nproj
  for (int e = threadIdx.x; e < nproj * nproj; e += kSThreads) qs[e] = q[e];
  __syncthreads();
  // workgroups are dealt to the 8 XCDs round-robin: consecutive rows (the
  // bands of one k) go to the same XCD
  const int bid = blockIdx.x;
  const int task = ((bid & 7) * per_xcd + (bid >> 3)) * (kSThreads / 64) + (int)(threadIdx.x >> 6);
  if (task >= ntask) return;
  const int k = task / nvec, r = task - k * nvec;
  if (r >= (cnt ? cnt[k] : nvec)) return;
  if (live && !live[task]) return;
  const int lane = threadIdx.x & 63;
  const long row = (long)k * kstride + (long)((off ? off[k] : 0) + r) * npwx;
  const cplx<T>* x = psi + row;
  cplx<T>* y = out + row;
  const int npw = npw_k[k];
  const cplx<T>* bk = beta + (long)k * nproj * npwx;
  constexpr int NC = NPL > 0 ? NPL : 1;
  cplx<T> xr[NC];
  if constexpr (NPL > 0) {
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int g = lane + 64 * i;
      xr[i] = g < npw ? x[g] : cplx<T>{T(0), T(0)};
    }
  }
  // lambda_p = sum_G conj(beta_p(G)) psi(G)   (Eq. lambdah), on every lane
  T lr[NP], li[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) lr[p] = li[p] = T(0);
  auto accumulate = [&](int g, const cplx<T>& xv) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (p < nproj) {
        const cplx<T> bv = bk[(long)p * npwx + g];
        lr[p] += bv.x * xv.x + bv.y * xv.y;
        li[p] += bv.x * xv.y - bv.y * xv.x;
      }
    }
  };
  if constexpr (NPL > 0) {
#pragma unroll
    for (int i = 0; i < NPL; ++i)
      if (lane + 64 * i < npw) accumulate(lane + 64 * i, xr[i]);
  } else {
    for (int g = lane; g < npw; g += 64) accumulate(g, x[g]);
  }
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    if (p < nproj) {
      lr[p] = wave_sum(lr[p]);
      li[p] = wave_sum(li[p]);
    }
  }
  // delta_p = sum_s q_ps lambda_s   (Eq. delta_eq), on every lane
  T dr[NP], di[NP];
#pragma unroll
  for (int p = 0; p < NP; ++p) {
    dr[p] = di[p] = T(0);
    if (p < nproj) {
#pragma unroll
      for (int s2 = 0; s2 < NP; ++s2) {
        if (s2 < nproj) {
          const cplx<T> qq = qs[p * nproj + s2];
          dr[p] += qq.x * lr[s2] - qq.y * li[s2];
          di[p] += qq.x * li[s2] + qq.y * lr[s2];
        }
      }
    }
  }
  // S psi = psi + sum_p delta_p beta_p   (Eq. finals)
  const T f = scale ? T(mult * scale[task]) : T(1);
  auto emit = [&](int g, cplx<T> v) {
    if (g >= npw) {
      if (!scale) y[g] = {T(0), T(0)};
      return;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (p < nproj) {
        const cplx<T> bv = bk[(long)p * npwx + g];
        v.x += dr[p] * bv.x - di[p] * bv.y;
        v.y += dr[p] * bv.y + di[p] * bv.x;
      }
    }
    if (scale) {
      const cplx<T> o = y[g];
      y[g] = {o.x + f * v.x, o.y + f * v.y};
    } else {
      y[g] = v;
    }
  };
  if constexpr (NPL > 0) {
#pragma unroll
    for (int i = 0; i < NPL; ++i)
      if (lane + 64 * i < npwx) emit(lane + 64 * i, xr[i]);
  } else {
    for (int g = lane; g < npwx; g += 64) emit(g, g < npw ? x[g] : cplx<T>{T(0), T(0)});
  }
}

// The projector rows of one k in LDS, read by all its bands: one workgroup per
// (k, group of up to kSBandsPerBlock rows).  Each row is handled by a half
// wavefront (32 lanes, two rows per wave at a time), which halves the cost of
// the lane reductions and of forming delta per row compared with a whole wave
// per row; each lane keeps its NPL plane waves (g = l + 32 i) of the row in
// registers.  Used when beta_k fits the LDS budget; it replaces the per-row
// L2 reads of beta (nproj rows per band, twice) by LDS reads.
constexpr int kSBandsPerBlock = 8;

// sum over the 32 lanes of each half of the wavefront, on every lane
template <class T>
__device__ __forceinline__ T half_sum(T v) {
  v += dpp<0xB1>(v);   // quad_perm 1,0,3,2
  v += dpp<0x4E>(v);   // quad_perm 2,3,0,1
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  return v;
}

template <class T, int NP, int NPL>
__global__ __launch_bounds__(kSThreads) void spsi_lds_kernel(const cplx<T>* psi, cplx<T>* out, long kstride,
                                                             int nvec, const int* __restrict__ off,
                                                             const int* __restrict__ cnt,
                                                             const int* __restrict__ live,
                                                             const int* __restrict__ npw_k, int npwx, int nproj,
                                                             const cplx<T>* __restrict__ beta,
                                                             const cplx<T>* __restrict__ q,
                                                             const double* __restrict__ scale, double mult,
                                                             int per_xcd, int ngroup, int groups_per_k) {
  extern __shared__ char smem[];
  auto* qs = reinterpret_cast<cplx<T>*>(smem);        // q, nproj x nproj
  cplx<T>* bs = qs + nproj * nproj;                   // beta_k, nproj x npw_k (row stride npwx)
  const int bid = blockIdx.x;
  const int grp = (bid & 7) * per_xcd + (bid >> 3);
  if (grp >= ngroup) return;                          // whole workgroup: no barrier skipped
  const int k = grp / groups_per_k;
  const int r0 = (grp - k * groups_per_k) * kSBandsPerBlock;
  const int nrow = min(kSBandsPerBlock, (cnt ? cnt[k] : nvec) - r0);
  if (nrow <= 0) return;
  const int npw = npw_k[k];
  const cplx<T>* bk = beta + (long)k * nproj * npwx;
  for (int e = threadIdx.x; e < nproj * nproj; e += kSThreads) qs[e] = q[e];
  for (int p = 0; p < nproj; ++p)
    for (int g = threadIdx.x; g < npw; g += kSThreads) bs[p * npwx + g] = bk[(long)p * npwx + g];
  __syncthreads();
  const int l = threadIdx.x & 31, half = threadIdx.x >> 5;
  // both halves of a wave run the same number of iterations (the row index
  // is clamped and the surplus half masked), so the lane sums see every lane
  constexpr int NH = kSThreads / 32;
  for (int rb = 0; rb < nrow; rb += NH) {
    const int rr = rb + half;
    const bool on = rr < nrow;
    const int r = r0 + (on ? rr : 0);
    const int task = k * nvec + r;
    const bool act = on && !(live && !live[task]);
    const long row = (long)k * kstride + (long)((off ? off[k] : 0) + r) * npwx;
    const cplx<T>* x = psi + row;
    cplx<T>* y = out + row;
    cplx<T> xr[NPL];
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int g = l + 32 * i;
      xr[i] = (act && g < npw) ? x[g] : cplx<T>{T(0), T(0)};
    }
    T lr[NP], li[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) lr[p] = li[p] = T(0);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int g = l + 32 * i;
      if (g < npw) {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          if (p < nproj) {
            const cplx<T> bv = bs[p * npwx + g];
            lr[p] += bv.x * xr[i].x + bv.y * xr[i].y;
            li[p] += bv.x * xr[i].y - bv.y * xr[i].x;
          }
        }
      }
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      if (p < nproj) {
        lr[p] = half_sum(lr[p]);
        li[p] = half_sum(li[p]);
      }
    }
    T dr[NP], di[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      dr[p] = di[p] = T(0);
      if (p < nproj) {
#pragma unroll
        for (int s2 = 0; s2 < NP; ++s2) {
          if (s2 < nproj) {
            const cplx<T> qq = qs[p * nproj + s2];
            dr[p] += qq.x * lr[s2] - qq.y * li[s2];
            di[p] += qq.x * li[s2] + qq.y * lr[s2];
          }
        }
      }
    }
    if (!act) continue;
    const T f = scale ? T(mult * scale[task]) : T(1);
#pragma unroll
    for (int i = 0; i < NPL; ++i) {
      const int g = l + 32 * i;
      if (g >= npwx) continue;
      if (g >= npw) {
        if (!scale) y[g] = {T(0), T(0)};
        continue;
      }
      cplx<T> v = xr[i];
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if (p < nproj) {
          const cplx<T> bv = bs[p * npwx + g];
          v.x += dr[p] * bv.x - di[p] * bv.y;
          v.y += dr[p] * bv.y + di[p] * bv.x;
        }
      }
      if (scale) {
        const cplx<T> o = y[g];
        y[g] = {o.x + f * v.x, o.y + f * v.y};
      } else {
        y[g] = v;
      }
    }
  }
}

constexpr size_t kSLdsBudget = 64 * 1024;

template <class T, int NP, int NPL>
void launch_spsi_t(pw_ctx* c, const VecSel& sel, const void* psi, void* out, const double* scale, double mult,
                   int nproj, const void* beta, const void* q, hipStream_t st) {
  if constexpr (NPL > 0) {
    const size_t lds_b = sizeof(cplx<T>) * ((size_t)nproj * nproj + (size_t)nproj * c->npwx);
    if (nproj > 0 && lds_b <= kSLdsBudget) {
      const int groups_per_k = (sel.nvec + kSBandsPerBlock - 1) / kSBandsPerBlock;
      const int ngroup = groups_per_k * c->nk;
      const int per_xcd = (ngroup + 7) / 8;
      hipLaunchKernelGGL((spsi_lds_kernel<T, NP, 2 * NPL>), dim3(8u * (unsigned)per_xcd), dim3(kSThreads), lds_b,
                         st, (const cplx<T>*)psi, (cplx<T>*)out, sel.kstride, sel.nvec, sel.off, sel.cnt, sel.live,
                         c->d_npw, c->npwx, nproj, (const cplx<T>*)beta, (const cplx<T>*)q, scale, mult, per_xcd,
                         ngroup, groups_per_k);
      return;
    }
  }
  const int ntask = sel.nvec * c->nk;
  const int nblk = (ntask + kSThreads / 64 - 1) / (kSThreads / 64);
  const int per_xcd = (nblk + 7) / 8;
  const size_t lds = sizeof(cplx<T>) * (size_t)std::max(1, nproj * nproj);
  hipLaunchKernelGGL((spsi_kernel<T, NP, NPL>), dim3(8u * (unsigned)per_xcd), dim3(kSThreads), lds, st,
                     (const cplx<T>*)psi, (cplx<T>*)out, sel.kstride, sel.nvec, sel.off, sel.cnt, sel.live, c->d_npw,
                     c->npwx, nproj, (const cplx<T>*)beta, (const cplx<T>*)q, scale, mult, per_xcd, ntask);
}

template <class T, int NP>
void launch_spsi_npl(pw_ctx* c, const VecSel& sel, const void* psi, void* out, const double* scale, double mult,
                     int nproj, const void* beta, const void* q, hipStream_t st) {
  const int chunks = (c->npwx + 63) / 64;
  if (chunks <= 2)
    launch_spsi_t<T, NP, 2>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
  else if (chunks <= 4)
    launch_spsi_t<T, NP, 4>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
  else if (chunks <= 6)
    launch_spsi_t<T, NP, 6>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
  else if (chunks <= 8)
    launch_spsi_t<T, NP, 8>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
  else if (chunks <= 12)
    launch_spsi_t<T, NP, 12>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
  else if (chunks <= 16)
    launch_spsi_t<T, NP, 16>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
  else
    launch_spsi_t<T, NP, 0>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
}

template <class T>
void launch_spsi_np(pw_ctx* c, const VecSel& sel, const void* psi, void* out, const double* scale, double mult,
                    int nproj, const void* beta, const void* q, hipStream_t st) {
  // up to 8 projectors (every workload here): rows held in registers; more:
  // one wave per row looping over the plane waves
  if (nproj <= 8)
    launch_spsi_npl<T, 8>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
  else
    launch_spsi_t<T, 32, 0>(c, sel, psi, out, scale, mult, nproj, beta, q, st);
}

}  // namespace

pw_status launch_spsi(pw_ctx* c, pw_prec prec, const VecSel& sel, const void* psi, void* out, const double* scale,
                      double mult, hipStream_t st) {
  if (sel.nvec <= 0) return PW_OK;
  const int nproj = c->have_q ? c->nproj : 0;
  if (nproj > kSMaxProj) return set_err(c, PW_EINVAL, "overlap: more than 32 projectors");
  if (prec == PW_FP64)
    launch_spsi_np<double>(c, sel, psi, out, scale, mult, nproj, c->d_beta64, c->d_q64, st);
  else
    launch_spsi_np<float>(c, sel, psi, out, scale, mult, nproj, c->d_beta32, c->d_q32, st);
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
