// Linear response at a wavevector q (Sec. 2.3; Algorithm phonon_new): the
// perturbed wavefunctions of k live on the k+q sphere, held by a second
// context whose k-point i is k_i + q on the same lattice, cutoff and mesh.
//
//   pw_dfpt_rhs:  rhs_nu = -(1 - S P_v^{k+q}) dV u_k nu   (Eq. linear_system,
//                 dS = 0), with (dV u)(G') = sum_G dV~[(m_G' - m_G) mod N] u(G)
//   pw_drho:      drho(r) = 4 sum_k w_k sum_nu conj(u_k nu(r)) du_k nu(r)
//                 (Eq. drho without the augmentation term)
//
// Both are formed in reciprocal space.  At these sphere sizes (npw ~ 300) the
// direct sum over the pairs (G', G) of the two spheres costs about 8 npw^2
// flop per band, less than the pruned FFT pair per band (~1 MFLOP at 24^3),
// and needs no mesh in memory:
//   * dV u is a per-k product of the npw_kq x npw_k matrix dV~[m' - m]
//     (gathered from the transformed perturbation, which stays in L2) with the
//     k's bands staged in LDS;
//   * drho accumulates, per k, M(G1, G2) = sum_nu conj(u(G1)) du(G2) (register
//     blocked over 4 x 4 pairs, bands staged in LDS) into bins of the Miller
//     difference d = m_G2 - m_G1 held in LDS; the per-k bins are summed over k
//     into the mesh (d mod N; 64 chunks of k summed in parallel, then the
//     chunks in a fixed order; the per-k bins themselves are summed with LDS
//     atomics, so results agree to rounding between runs, not bit for bit)
//     and one inverse transform of the mesh gives
//     drho(r) = sum_d F(d) exp(2 pi i d.l / N).
// The transforms of the single mesh (dV(r) -> dV~ with 1/N_r, F -> drho(r))
// are separable direct sums, one launch per axis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "host_util.hpp"
#include "internal.hpp"

namespace mkpw {

using cd = cplx<double>;

namespace {

__device__ __forceinline__ void unpack_miller(int key, int& a, int& b, int& c) {
  a = ((key >> 20) & 1023) - 512;
  b = ((key >> 10) & 1023) - 512;
  c = (key & 1023) - 512;
}

__device__ __forceinline__ int wrap(int d, int n) {
  d %= n;
  return d < 0 ? d + n : d;
}

// one axis of a separable DFT of the n1 x n2 x n3 mesh (C order, l3 fastest):
// out(.., l, ..) = scale * sum_j in(.., j, ..) exp(sign 2 pi i j l / n_axis)
__global__ __launch_bounds__(256) void mesh_dft_axis_kernel(const cd* __restrict__ in, cd* __restrict__ out, int n1,
                                                            int n2, int n3, int axis, int sign, double scale) {
  const long total = (long)n1 * n2 * n3;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int l3 = (int)(e % n3), l2 = (int)((e / n3) % n2), l1 = (int)(e / ((long)n2 * n3));
  const int n = axis == 0 ? n1 : axis == 1 ? n2 : n3;
  const int l = axis == 0 ? l1 : axis == 1 ? l2 : l3;
  const long stride = axis == 0 ? (long)n2 * n3 : axis == 1 ? n3 : 1;
  const long base = e - (long)l * stride;
  double sr = 0.0, si = 0.0;
  for (int j = 0; j < n; ++j) {
    const int t = (int)(((long)j * l) % n);
    double s, c;
    sincospi(2.0 * t / n, &s, &c);
    s *= sign;
    const cd v = in[base + (long)j * stride];
    sr += v.x * c - v.y * s;
    si += v.x * s + v.y * c;
  }
  out[e] = {scale * sr, scale * si};
}

constexpr int kVT = 128;  // output plane waves per workgroup
constexpr int kVG = 64;   // input plane waves staged per step
constexpr int kVB = 16;   // bands per pass

// out(k, b, G') = scale * sum_G dvt[(m_G' - m_G) mod N] psi(k, b, G)
__global__ __launch_bounds__(kVT) void dvpsi_kernel(const cd* __restrict__ dvt, int n1, int n2, int n3,
                                                    const int* __restrict__ npw_in, const int* __restrict__ key_in,
                                                    int npwx_in, const cd* __restrict__ psi,
                                                    const int* __restrict__ npw_out, const int* __restrict__ key_out,
                                                    int npwx_out, cd* __restrict__ out, int nbnd, double scale) {
  const int k = blockIdx.y;
  const int gp = blockIdx.x * kVT + threadIdx.x;
  const int nin = npw_in[k], nout = npw_out[k];
  __shared__ cd us[kVB][kVG];
  __shared__ int ms[3][kVG];
  // mesh index of m_G' - m_G on each axis as (m_G' mod n) + (-m_G mod n),
  // both in [0, n), less n when the sum reaches n: no division per pair
  int p1 = 0, p2 = 0, p3 = 0;
  if (gp < nout) unpack_miller(key_out[(long)k * npwx_out + gp], p1, p2, p3);
  p1 = wrap(p1, n1);
  p2 = wrap(p2, n2);
  p3 = wrap(p3, n3);
  for (int b0 = 0; b0 < nbnd; b0 += kVB) {
    double ar[kVB], ai[kVB];
#pragma unroll
    for (int b = 0; b < kVB; ++b) ar[b] = ai[b] = 0.0;
    for (int g0 = 0; g0 < nin; g0 += kVG) {
      __syncthreads();
      for (int e = threadIdx.x; e < kVB * kVG; e += kVT) {
        const int b = e / kVG, g = e % kVG;
        us[b][g] = (b0 + b < nbnd && g0 + g < nin) ? psi[((long)k * nbnd + b0 + b) * npwx_in + g0 + g] : cd{0.0, 0.0};
      }
      for (int g = threadIdx.x; g < kVG; g += kVT) {
        int a = 0, b = 0, c = 0;
        if (g0 + g < nin) unpack_miller(key_in[(long)k * npwx_in + g0 + g], a, b, c);
        ms[0][g] = wrap(-a, n1);
        ms[1][g] = wrap(-b, n2);
        ms[2][g] = wrap(-c, n3);
      }
      __syncthreads();
      if (gp < nout) {
        const int ng = min(kVG, nin - g0);
        for (int g = 0; g < ng; ++g) {
          int d1 = p1 + ms[0][g], d2 = p2 + ms[1][g], d3 = p3 + ms[2][g];
          d1 -= d1 >= n1 ? n1 : 0;
          d2 -= d2 >= n2 ? n2 : 0;
          d3 -= d3 >= n3 ? n3 : 0;
          const int idx = (d1 * n2 + d2) * n3 + d3;
          const cd v = dvt[idx];
#pragma unroll
          for (int b = 0; b < kVB; ++b) {
            const cd u = us[b][g];
            ar[b] += v.x * u.x - v.y * u.y;
            ai[b] += v.x * u.y + v.y * u.x;
          }
        }
      }
    }
    if (gp < npwx_out) {
      for (int b = 0; b < kVB && b0 + b < nbnd; ++b) {
        cd o = {0.0, 0.0};
        if (gp < nout) o = {scale * ar[b], scale * ai[b]};
        out[((long)k * nbnd + b0 + b) * npwx_out + gp] = o;
      }
    }
  }
}

constexpr int kRT = 64;    // plane waves of each sphere per pair tile
constexpr int kRB = 16;    // bands staged per step
constexpr int kRW = 1024;  // work-items per k-point: a 32 x 32 grid of 2 x 2 pair blocks

// Per k: bins F_k(d) += 4 w_k sum_nu conj(u1(G1)) u2(G2) over the pairs with
// d = m_G2 - m_G1 - org_k in the box [0, D1) x [0, D2) x [0, D3), for the
// slice x0 <= d1 < x0 + nx held in LDS; the slice is written to part[k].
// The bins fill most of the LDS, so one workgroup runs per CU: it has 16
// waves, each work-item summing a 2 x 2 block of pairs of the 64 x 64 tile
// over the bands staged in LDS, so that enough waves hide the LDS latency.
// The bins are summed with LDS atomics: the order of the additions into a bin
// varies from run to run (results agree to rounding, not bit for bit).
__global__ __launch_bounds__(kRW) void drho_pairs_kernel(int nbnd, const double* __restrict__ wk,
                                                         const int* __restrict__ npw1, const int* __restrict__ key1,
                                                         int npwx1, const cd* __restrict__ u1,
                                                         const int* __restrict__ npw2, const int* __restrict__ key2,
                                                         int npwx2, const cd* __restrict__ u2,
                                                         const int* __restrict__ org, int D1, int D2, int D3, int x0,
                                                         int nx, cd* __restrict__ part) {
  extern __shared__ char smem[];
  const int nbin = nx * D2 * D3;
  const int nbin_al = (nbin + 1) & ~1;  // keeps the complex tiles 16-byte aligned
  double* bre = reinterpret_cast<double*>(smem);
  double* bim = bre + nbin_al;
  cd* us = reinterpret_cast<cd*>(bim + nbin_al);  // [kRB][kRT]
  cd* vs = us + kRB * kRT;                     // [kRB][kRT]
  int* ma = reinterpret_cast<int*>(vs + kRB * kRT);  // [3][kRT]
  int* mb = ma + 3 * kRT;                            // [3][kRT]
  const int k = blockIdx.x;
  for (int e = threadIdx.x; e < nbin; e += kRW) bre[e] = bim[e] = 0.0;
  const int n1 = npw1[k], n2 = npw2[k];
  const double f = 4.0 * wk[k];
  const int o1 = org[3 * k], o2 = org[3 * k + 1], o3 = org[3 * k + 2];
  constexpr int kBl = 2;  // pairs per work-item along each sphere
  const int ti = threadIdx.x >> 5, tj = threadIdx.x & 31;
  for (int i0 = 0; i0 < n1; i0 += kRT) {
    for (int j0 = 0; j0 < n2; j0 += kRT) {
      double cr[kBl][kBl], ci[kBl][kBl];
#pragma unroll
      for (int a = 0; a < kBl; ++a)
#pragma unroll
        for (int c = 0; c < kBl; ++c) cr[a][c] = ci[a][c] = 0.0;
      for (int b0 = 0; b0 < nbnd; b0 += kRB) {
        __syncthreads();
        for (int e = threadIdx.x; e < kRB * kRT; e += kRW) {
          const int b = e / kRT, g = e % kRT;
          const bool bok = b0 + b < nbnd;
          us[e] = (bok && i0 + g < n1) ? u1[((long)k * nbnd + b0 + b) * npwx1 + i0 + g] : cd{0.0, 0.0};
          vs[e] = (bok && j0 + g < n2) ? u2[((long)k * nbnd + b0 + b) * npwx2 + j0 + g] : cd{0.0, 0.0};
        }
        if (b0 == 0) {
          for (int g = threadIdx.x; g < kRT; g += kRW) {
            int a = 0, b = 0, c = 0;
            if (i0 + g < n1) unpack_miller(key1[(long)k * npwx1 + i0 + g], a, b, c);
            ma[g] = a;
            ma[kRT + g] = b;
            ma[2 * kRT + g] = c;
            a = b = c = 0;
            if (j0 + g < n2) unpack_miller(key2[(long)k * npwx2 + j0 + g], a, b, c);
            mb[g] = a;
            mb[kRT + g] = b;
            mb[2 * kRT + g] = c;
          }
        }
        __syncthreads();
#pragma unroll 4
        for (int b = 0; b < kRB; ++b) {
          cd x[kBl], y[kBl];
#pragma unroll
          for (int a = 0; a < kBl; ++a) x[a] = us[b * kRT + ti * kBl + a];
#pragma unroll
          for (int c = 0; c < kBl; ++c) y[c] = vs[b * kRT + tj * kBl + c];
#pragma unroll
          for (int a = 0; a < kBl; ++a)
#pragma unroll
            for (int c = 0; c < kBl; ++c) {
              // conj(x) * y
              cr[a][c] += x[a].x * y[c].x + x[a].y * y[c].y;
              ci[a][c] += x[a].x * y[c].y - x[a].y * y[c].x;
            }
        }
      }
      // scatter the 2 x 2 block into the bins of this slice
#pragma unroll
      for (int a = 0; a < kBl; ++a) {
        const int g1 = ti * kBl + a;
        if (i0 + g1 >= n1) continue;
#pragma unroll
        for (int c = 0; c < kBl; ++c) {
          const int g2 = tj * kBl + c;
          if (j0 + g2 >= n2) continue;
          const int d1 = mb[g2] - ma[g1] - o1 - x0;
          if (d1 < 0 || d1 >= nx) continue;
          const int d2 = mb[kRT + g2] - ma[kRT + g1] - o2;
          const int d3 = mb[2 * kRT + g2] - ma[2 * kRT + g1] - o3;
          const int bin = (d1 * D2 + d2) * D3 + d3;
          atomicAdd(&bre[bin], f * cr[a][c]);
          atomicAdd(&bim[bin], f * ci[a][c]);
        }
      }
    }
  }
  __syncthreads();
  cd* dst = part + ((long)k * D1 + x0) * D2 * D3;
  for (int e = threadIdx.x; e < nbin; e += kRW) dst[e] = {bre[e], bim[e]};
}

// F_c(l) = sum over the k of chunk c (k = c, c + nchunk, ...) of the part[k]
// bins b with (org_k + b) = l (mod N) on every axis; then F = sum_c F_c in a
// fixed order (no atomics in this reduction)
__global__ __launch_bounds__(256) void drho_reduce_kernel(const cd* __restrict__ part, const int* __restrict__ org,
                                                          int nk, int nchunk, int D1, int D2, int D3, int n1, int n2,
                                                          int n3, cd* __restrict__ Fc) {
  const long total = (long)n1 * n2 * n3;
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  const int c = blockIdx.y;
  const int l3 = (int)(e % n3), l2 = (int)((e / n3) % n2), l1 = (int)(e / ((long)n2 * n3));
  double sr = 0.0, si = 0.0;
  for (int k = c; k < nk; k += nchunk) {
    const cd* pk = part + (long)k * D1 * D2 * D3;
    for (int b1 = wrap(l1 - org[3 * k], n1); b1 < D1; b1 += n1)
      for (int b2 = wrap(l2 - org[3 * k + 1], n2); b2 < D2; b2 += n2)
        for (int b3 = wrap(l3 - org[3 * k + 2], n3); b3 < D3; b3 += n3) {
          const cd v = pk[((long)b1 * D2 + b2) * D3 + b3];
          sr += v.x;
          si += v.y;
        }
  }
  Fc[(long)c * total + e] = {sr, si};
}

__global__ __launch_bounds__(256) void sum_chunks_kernel(const cd* __restrict__ Fc, int nchunk, long total,
                                                         cd* __restrict__ F) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= total) return;
  double sr = 0.0, si = 0.0;
  for (int c = 0; c < nchunk; ++c) {
    sr += Fc[(long)c * total + e].x;
    si += Fc[(long)c * total + e].y;
  }
  F[e] = {sr, si};
}

// ctx_k and ctx_kq describe the same crystal on the same device: lattice,
// cutoff, mesh and number of k-points equal
pw_status check_pair(pw_ctx* ckq, const pw_ctx* ck) {
  if (!ckq || !ck) return PW_EINVAL;
  if (ckq->host_only || ck->host_only) return set_err(ckq, PW_ESTATE, "host-only context runs no device work");
  if (!ckq->have_k || !ck->have_k) return set_err(ckq, PW_ESTATE, "set k-points on both contexts first");
  if (ckq->device != ck->device) return set_err(ckq, PW_EINVAL, "the two contexts are on different devices");
  if (ckq->nk != ck->nk) return set_err(ckq, PW_EINVAL, "the two contexts hold different numbers of k-points");
  for (int i = 0; i < 3; ++i)
    if (ckq->fft[i] != ck->fft[i]) return set_err(ckq, PW_EINVAL, "the two contexts use different FFT meshes");
  for (int i = 0; i < 9; ++i)
    if (ckq->lat[i] != ck->lat[i]) return set_err(ckq, PW_EINVAL, "the two contexts use different lattices");
  return PW_OK;
}

// dV~ = forward transform of dV(r) with 1/N_r (Eq. fwFFT), on the device
pw_status transform_dv(pw_ctx* c, const double* dv_host, cd* dvt, cd* tmp, hipStream_t st) {
  const int n1 = c->fft[0], n2 = c->fft[1], n3 = c->fft[2];
  const long nr = (long)n1 * n2 * n3;
  MKPW_HIP(c, hipMemcpyAsync(tmp, dv_host, sizeof(cd) * nr, hipMemcpyHostToDevice, st));
  const dim3 grid((unsigned)((nr + 255) / 256));
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, tmp, dvt, n1, n2, n3, 0, -1, 1.0);
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, dvt, tmp, n1, n2, n3, 1, -1, 1.0);
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, tmp, dvt, n1, n2, n3, 2, -1, 1.0 / (double)nr);
  MKPW_TRY(check_launch(c, "mesh_dft", st));
  // the host array must stay readable until the copy has run
  MKPW_HIP(c, hipStreamSynchronize(st));
  return PW_OK;
}

}  // namespace

}  // namespace mkpw

extern "C" pw_status pw_dfpt_rhs(pw_ctx* ckq, const pw_ctx* ck, int nocc, const void* dv_r, const void* psi_k,
                                 const void* psi_occ_kq, void* rhs) {
  using namespace mkpw;
  MKPW_TRY(check_pair(ckq, ck));
  if (!dv_r || !psi_k || !psi_occ_kq || !rhs) return set_err(ckq, PW_EINVAL, "null argument");
  if (nocc < 1 || nocc > 64) return set_err(ckq, PW_EINVAL, "nocc must be in [1, 64]");
  (void)hipSetDevice(ckq->device);
  hipStream_t st = ckq->stream;
  const int nk = ckq->nk;
  const long nr = (long)ckq->fft[0] * ckq->fft[1] * ckq->fft[2];
  DevBufs b(ckq);
  cd *dvt, *tmp, *W;
  MKPW_TRY(b.get((size_t)nr, &dvt));
  MKPW_TRY(b.get((size_t)nr, &tmp));
  MKPW_TRY(b.get((size_t)nk * nocc * nocc, &W));
  MKPW_TRY(transform_dv(ckq, (const double*)dv_r, dvt, tmp, st));
  // rhs0 = -dV u (on the k+q sphere)
  {
    const dim3 grid((unsigned)((ckq->npwx + kVT - 1) / kVT), (unsigned)nk);
    hipLaunchKernelGGL(dvpsi_kernel, grid, dim3(kVT), 0, st, dvt, ckq->fft[0], ckq->fft[1], ckq->fft[2], ck->d_npw,
                       ck->d_mkey, ck->npwx, (const cd*)psi_k, ckq->d_npw, ckq->d_mkey, ckq->npwx, (cd*)rhs, nocc,
                       -1.0);
    MKPW_TRY(check_launch(ckq, "dvpsi", st));
  }
  // rhs = rhs0 - S U (U^H rhs0)  =  -(1 - S P_v) dV u
  const cd* U = (const cd*)psi_occ_kq;
  const cd* P = U;
  if (ckq->have_q) {
    cd* SU;
    MKPW_TRY(b.get((size_t)nk * nocc * ckq->npwx, &SU));
    VecSel sel;
    sel.nvec = nocc;
    sel.kstride = (long)nocc * ckq->npwx;
    MKPW_TRY(launch_spsi(ckq, PW_FP64, sel, U, SU, nullptr, 0.0, st));
    P = SU;
  }
  GramArgs g;
  g.A = U; g.a_kstride = (long)nocc * ckq->npwx; g.a_n = nocc;
  g.B = (const cd*)rhs; g.b_kstride = (long)nocc * ckq->npwx; g.b_n = nocc;
  g.ld = ckq->npwx; g.npw = ckq->d_npw;
  g.C = W; g.c_kstride = (long)nocc * nocc; g.ldc = nocc;
  MKPW_TRY(launch_gram(ckq, g, nocc, nocc, st));
  CombArgs m;
  m.X = P; m.x_kstride = (long)nocc * ckq->npwx; m.x_n = nocc;
  m.Y = (cd*)rhs; m.y_kstride = (long)nocc * ckq->npwx; m.y_n = nocc;
  m.ld = ckq->npwx; m.Cm = W; m.c_kstride = (long)nocc * nocc; m.ldc = nocc;
  m.alpha = -1.0; m.accumulate = 1;
  MKPW_TRY(launch_combine(ckq, m, nocc, st));
  MKPW_HIP(ckq, hipStreamSynchronize(st));
  return PW_OK;
}

extern "C" pw_status pw_drho(pw_ctx* ckq, const pw_ctx* ck, int nbnd, const double* wk, const void* psi_k,
                             const void* dpsi_kq, void* drho_r) {
  using namespace mkpw;
  MKPW_TRY(check_pair(ckq, ck));
  if (!wk || !psi_k || !dpsi_kq || !drho_r) return set_err(ckq, PW_EINVAL, "null argument");
  if (nbnd < 1 || nbnd > 1024) return set_err(ckq, PW_EINVAL, "nbnd must be in [1, 1024]");
  (void)hipSetDevice(ckq->device);
  hipStream_t st = ckq->stream;
  const int nk = ckq->nk;
  const int n1 = ckq->fft[0], n2 = ckq->fft[1], n3 = ckq->fft[2];
  const long nr = (long)n1 * n2 * n3;
  // per-k origin of the Miller difference m(k+q) - m(k) and the common box
  std::vector<int> org(3 * (size_t)nk);
  int D[3] = {1, 1, 1};
  for (int k = 0; k < nk; ++k) {
    for (int a = 0; a < 3; ++a) {
      int lo1 = 1 << 20, hi1 = -(1 << 20), lo2 = 1 << 20, hi2 = -(1 << 20);
      for (int g = 0; g < ck->npw[k]; ++g) {
        const int v = ck->miller[((size_t)k * ck->npwx + g) * 3 + a];
        lo1 = std::min(lo1, v);
        hi1 = std::max(hi1, v);
      }
      for (int g = 0; g < ckq->npw[k]; ++g) {
        const int v = ckq->miller[((size_t)k * ckq->npwx + g) * 3 + a];
        lo2 = std::min(lo2, v);
        hi2 = std::max(hi2, v);
      }
      org[3 * k + a] = lo2 - hi1;
      D[a] = std::max(D[a], hi2 - lo1 - (lo2 - hi1) + 1);
    }
  }
  // LDS: bins of a slice of the box, the two band tiles and the Miller tiles
  const size_t tiles = 2 * sizeof(cd) * kRB * kRT + 6 * sizeof(int) * kRT;
  const size_t lds_max = 150 * 1024;
  const size_t per_x = 2 * sizeof(double) * (size_t)D[1] * D[2];
  if (per_x + tiles + 2 * sizeof(double) > lds_max) return set_err(ckq, PW_EINVAL, "drho: plane-wave spheres too large for the bins");
  const int nx = (int)std::min<size_t>(D[0], (lds_max - tiles - 2 * sizeof(double)) / per_x);
  DevBufs b(ckq);
  cd *part, *F, *tmp, *Fc;
  int* d_org;
  double* d_w;
  const int nchunk = std::min(nk, 64);
  MKPW_TRY(b.get((size_t)nk * D[0] * D[1] * D[2], &part));
  MKPW_TRY(b.get((size_t)nchunk * nr, &Fc));
  MKPW_TRY(b.get((size_t)nr, &F));
  MKPW_TRY(b.get((size_t)nr, &tmp));
  MKPW_TRY(b.get((size_t)3 * nk, &d_org));
  MKPW_TRY(b.get((size_t)nk, &d_w));
  MKPW_HIP(ckq, hipMemcpyAsync(d_org, org.data(), sizeof(int) * org.size(), hipMemcpyHostToDevice, st));
  MKPW_HIP(ckq, hipMemcpyAsync(d_w, wk, sizeof(double) * nk, hipMemcpyHostToDevice, st));
  for (int x0 = 0; x0 < D[0]; x0 += nx) {
    const int nxx = std::min(nx, D[0] - x0);
    const size_t lds = per_x * nxx + tiles + 2 * sizeof(double);
    MKPW_TRY(ensure_lds_limit(ckq, (const void*)drho_pairs_kernel, lds));
    hipLaunchKernelGGL(drho_pairs_kernel, dim3((unsigned)nk), dim3(kRW), lds, st, nbnd, d_w, ck->d_npw, ck->d_mkey,
                       ck->npwx, (const cd*)psi_k, ckq->d_npw, ckq->d_mkey, ckq->npwx, (const cd*)dpsi_kq, d_org,
                       D[0], D[1], D[2], x0, nxx, part);
    MKPW_TRY(check_launch(ckq, "drho_pairs", st));
  }
  const dim3 grid((unsigned)((nr + 255) / 256));
  hipLaunchKernelGGL(drho_reduce_kernel, dim3(grid.x, (unsigned)nchunk), dim3(256), 0, st, part, d_org, nk, nchunk,
                     D[0], D[1], D[2], n1, n2, n3, Fc);
  hipLaunchKernelGGL(sum_chunks_kernel, grid, dim3(256), 0, st, Fc, nchunk, nr, F);
  // drho(r) = sum_f F(f) exp(+2 pi i f.l / N)
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, F, tmp, n1, n2, n3, 0, 1, 1.0);
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, tmp, F, n1, n2, n3, 1, 1, 1.0);
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, F, (cd*)drho_r, n1, n2, n3, 2, 1, 1.0);
  MKPW_TRY(check_launch(ckq, "drho", st));
  MKPW_HIP(ckq, hipStreamSynchronize(st));
  return PW_OK;
}
