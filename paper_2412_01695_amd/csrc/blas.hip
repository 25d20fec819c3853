// Small batched complex FP64 linear algebra over ragged per-k blocks of rows.
//
// Wavefunction blocks are rows of length npwx (one row per vector, (nk, nvec,
// npwx) layout).  The Davidson and CG solvers need, per k-point:
//   gram:         C = A^H B           (inner products of two row blocks)
//   rows_combine: Y = beta Y + alpha X^T-combination  Y_j = sum_i X_i c_ij
//   rows_trmm:    in-place Y <- Y M with M upper triangular
//   conversions between complex128 and complex64 rows.
// Every k-point has its own row offsets and counts (device arrays), so k-points
// at different stages of a solve share one launch; a count of zero idles a k.
#include <hip/hip_runtime.h>

#include "fft.hpp"
#include "internal.hpp"

namespace mkpw {

using c64d = cplx<double>;

__device__ __forceinline__ int sel_i(const int* p, int k, int dflt) { return p ? p[k] : dflt; }

// ------------------------------------------------------------------ gram: C = A^H B

constexpr int kGT = 16;   // output tile
constexpr int kGK = 32;   // k-chunk (plane waves) staged in LDS

__global__ __launch_bounds__(256) void gram_kernel(GramArgs a) {
  const int k = blockIdx.x;
  const int ni = sel_i(a.a_cnt, k, a.a_n);
  const int nj = sel_i(a.b_cnt, k, a.b_n);
  const int i0 = blockIdx.y * kGT, j0 = blockIdx.z * kGT;
  if (i0 >= ni || j0 >= nj) return;
  if (a.b_live) {  // a tile none of whose B vectors takes part is skipped
    const int* lv = a.b_live + (long)k * a.live_kstride;
    bool any = false;
    for (int j = j0; j < min(j0 + kGT, nj); ++j) any |= lv[j] != 0;
    if (!any) return;
  }
  const int npw = a.npw[k];
  const c64d* A = a.A + (long)k * a.a_kstride + (long)sel_i(a.a_off, k, a.a_row) * a.ld;
  const c64d* B = a.B + (long)k * a.b_kstride + (long)sel_i(a.b_off, k, a.b_row) * a.ld;
  __shared__ c64d As[kGT][kGK + 1];
  __shared__ c64d Bs[kGT][kGK + 1];
  const int tid = threadIdx.x;
  const int ti = tid / kGT, tj = tid % kGT;
  double sr = 0.0, si = 0.0;
  // each work-item stages kGT * kGK / 256 = 2 elements of each tile; the next
  // chunk's elements are loaded into registers while the current one is used
  constexpr int kPer = kGT * kGK / 256;
  c64d na[kPer], nb[kPer];
  auto fetch = [&](int g0) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * 256, r = e / kGK, g = e % kGK;
      na[q] = nb[q] = c64d{0.0, 0.0};
      if (g0 + g < npw) {
        if (i0 + r < ni) na[q] = A[(long)(i0 + r) * a.ld + g0 + g];
        if (j0 + r < nj) nb[q] = B[(long)(j0 + r) * a.ld + g0 + g];
      }
    }
  };
  fetch(0);
  for (int g0 = 0; g0 < npw; g0 += kGK) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int e = tid + q * 256, r = e / kGK, g = e % kGK;
      As[r][g] = na[q];
      Bs[r][g] = nb[q];
    }
    __syncthreads();
    if (g0 + kGK < npw) fetch(g0 + kGK);
#pragma unroll 8
    for (int g = 0; g < kGK; ++g) {
      c64d x = As[ti][g], y = Bs[tj][g];
      sr += x.x * y.x + x.y * y.y;
      si += x.x * y.y - x.y * y.x;
    }
    __syncthreads();
  }
  const int i = i0 + ti, j = j0 + tj;
  if (i < ni && j < nj && (!a.b_live || a.b_live[(long)k * a.live_kstride + j])) {
    c64d* C = a.C + (long)k * a.c_kstride;
    const int r = sel_i(a.c_roff, k, a.c_row) + i, c = sel_i(a.c_coff, k, a.c_col) + j;
    double vr = a.alpha * sr, vi = a.alpha * si;
    C[(long)r * a.ldc + c] = {vr, vi};
    // mirrored entry, unless that position is itself computed directly
    const int r0 = sel_i(a.c_roff, k, a.c_row), c0 = sel_i(a.c_coff, k, a.c_col);
    if (a.mirror && !(c >= r0 && c < r0 + ni && r >= c0 && r < c0 + nj)) C[(long)c * a.ldc + r] = {vr, -vi};
  }
}

// ------------------------------------------------------------------ rows_combine

constexpr int kRJ = 8;  // output rows per pass

__global__ __launch_bounds__(256) void rows_combine_kernel(CombArgs a) {
  const int k = blockIdx.y;
  const int ni = sel_i(a.x_cnt, k, a.x_n);
  const int nj = sel_i(a.y_cnt, k, a.y_n);
  if (nj <= 0) return;
  const int npwx = a.ld;
  const int g = blockIdx.x * 256 + threadIdx.x;
  const c64d* X = a.X + (long)k * a.x_kstride + (long)sel_i(a.x_off, k, a.x_row) * npwx;
  c64d* Y = a.Y + (long)k * a.y_kstride + (long)sel_i(a.y_off, k, a.y_row) * npwx;
  const c64d* Cm = a.Cm + (long)k * a.c_kstride + (long)sel_i(a.c_roff, k, a.c_row) * a.ldc +
                   sel_i(a.c_coff, k, a.c_col);
  __shared__ c64d cs[64][kRJ];
  const int* lv = a.y_live ? a.y_live + (long)k * a.live_kstride : nullptr;
  for (int j0 = 0; j0 < nj; j0 += kRJ) {
    if (lv) {  // a pass none of whose output rows takes part is skipped (uniform over the block)
      bool any = false;
      for (int jj = j0; jj < min(j0 + kRJ, nj); ++jj) any |= lv[jj] != 0;
      if (!any) continue;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < ni * kRJ; e += 256) {
      int i = e / kRJ, jj = e % kRJ;
      cs[i][jj] = (j0 + jj < nj) ? Cm[(long)i * a.ldc + j0 + jj] : c64d{0.0, 0.0};
    }
    __syncthreads();
    if (g >= npwx) continue;
    double ar[kRJ], ai[kRJ];
#pragma unroll
    for (int jj = 0; jj < kRJ; ++jj) ar[jj] = ai[jj] = 0.0;
    for (int i = 0; i < ni; ++i) {
      c64d x = X[(long)i * npwx + g];
#pragma unroll
      for (int jj = 0; jj < kRJ; ++jj) {
        c64d c = cs[i][jj];
        ar[jj] += x.x * c.x - x.y * c.y;
        ai[jj] += x.x * c.y + x.y * c.x;
      }
    }
#pragma unroll
    for (int jj = 0; jj < kRJ; ++jj) {
      if (j0 + jj < nj && (!lv || lv[j0 + jj])) {
        c64d* y = Y + (long)(j0 + jj) * npwx + g;
        c64d o = a.accumulate ? *y : c64d{0.0, 0.0};
        *y = {o.x + a.alpha * ar[jj], o.y + a.alpha * ai[jj]};
      }
    }
  }
}

// ------------------------------------------------------------------ in-place Y <- Y M, M upper triangular

__global__ __launch_bounds__(256) void rows_trmm_kernel(c64d* Yb, long y_kstride, const int* y_off, const int* y_cnt,
                                                        int npwx, const c64d* Mb, long m_kstride, int ldm) {
  const int k = blockIdx.y;
  const int n = y_cnt[k];
  if (n <= 0) return;
  const int g = blockIdx.x * 256 + threadIdx.x;
  c64d* Y = Yb + (long)k * y_kstride + (long)y_off[k] * npwx;
  const c64d* M = Mb + (long)k * m_kstride;
  __shared__ c64d ms[32 * 32];
  for (int e = threadIdx.x; e < n * n; e += 256) ms[e] = M[(long)(e / n) * ldm + (e % n)];
  __syncthreads();
  if (g >= npwx) return;
  // each row of this work-item's column is read once and added into the
  // outputs it feeds (Y_j = sum_{i <= j} Y_i M_ij, outputs in registers)
  constexpr int kMax = 32;
  double ar[kMax], ai[kMax];
#pragma unroll
  for (int j = 0; j < kMax; ++j) ar[j] = ai[j] = 0.0;
  for (int i = 0; i < n; ++i) {
    const c64d x = Y[(long)i * npwx + g];
#pragma unroll
    for (int j = 0; j < kMax; ++j) {
      if (j >= i && j < n) {
        const c64d c = ms[i * n + j];
        ar[j] += x.x * c.x - x.y * c.y;
        ai[j] += x.x * c.y + x.y * c.x;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < kMax; ++j)
    if (j < n) Y[(long)j * npwx + g] = {ar[j], ai[j]};
}

// ------------------------------------------------------------------ precision conversion of row blocks

// (with `live`, row v of k is converted only if live[k * nvec + v])
__global__ void rows_to_c64_kernel(const c64d* __restrict__ src, long s_kstride, const int* s_off,
                                   cplx<float>* __restrict__ dst, long d_kstride, const int* d_off, const int* cnt,
                                   int nvec, int npwx, const int* live) {
  const int k = blockIdx.y;
  const int n = cnt ? cnt[k] : nvec;
  const long total = (long)n * npwx;
  const c64d* s = src + (long)k * s_kstride + (long)(s_off ? s_off[k] : 0) * npwx;
  cplx<float>* d = dst + (long)k * d_kstride + (long)(d_off ? d_off[k] : 0) * npwx;
  const int* lv = live ? live + (long)k * nvec : nullptr;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    if (!lv || lv[e / npwx]) d[e] = {(float)s[e].x, (float)s[e].y};
}

__global__ void rows_to_c128_kernel(const cplx<float>* __restrict__ src, long s_kstride, const int* s_off,
                                    c64d* __restrict__ dst, long d_kstride, const int* d_off, const int* cnt,
                                    int nvec, int npwx, const int* live) {
  const int k = blockIdx.y;
  const int n = cnt ? cnt[k] : nvec;
  const long total = (long)n * npwx;
  const cplx<float>* s = src + (long)k * s_kstride + (long)(s_off ? s_off[k] : 0) * npwx;
  c64d* d = dst + (long)k * d_kstride + (long)(d_off ? d_off[k] : 0) * npwx;
  const int* lv = live ? live + (long)k * nvec : nullptr;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x)
    if (!lv || lv[e / npwx]) d[e] = {(double)s[e].x, (double)s[e].y};
}

// ------------------------------------------------------------------ host launchers

pw_status launch_gram(pw_ctx* c, const GramArgs& a, int ni_max, int nj_max, hipStream_t st) {
  if (ni_max <= 0 || nj_max <= 0) return PW_OK;
  dim3 grid(c->nk, (ni_max + kGT - 1) / kGT, (nj_max + kGT - 1) / kGT);
  hipLaunchKernelGGL(gram_kernel, grid, dim3(256), 0, st, a);
  return check_launch(c, "gram", st);
}

pw_status launch_combine(pw_ctx* c, const CombArgs& a, int ni_max, hipStream_t st) {
  if (ni_max > 64) return set_err(c, PW_EINVAL, "rows_combine: more than 64 input rows");
  dim3 grid((a.ld + 255) / 256, c->nk);
  hipLaunchKernelGGL(rows_combine_kernel, grid, dim3(256), 0, st, a);
  return check_launch(c, "rows_combine", st);
}

pw_status launch_trmm(pw_ctx* c, cplx<double>* Y, long y_kstride, const int* y_off, const int* y_cnt,
                      const cplx<double>* M, long m_kstride, int ldm, hipStream_t st) {
  dim3 grid((c->npwx + 255) / 256, c->nk);
  hipLaunchKernelGGL(rows_trmm_kernel, grid, dim3(256), 0, st, Y, y_kstride, y_off, y_cnt, c->npwx, M, m_kstride,
                     ldm);
  return check_launch(c, "rows_trmm", st);
}

pw_status launch_to_c64(pw_ctx* c, const cplx<double>* src, long s_kstride, const int* s_off, cplx<float>* dst,
                        long d_kstride, const int* d_off, const int* cnt, int nvec, hipStream_t st, const int* live) {
  dim3 grid(std::max(1, std::min(64, (nvec * c->npwx + 255) / 256)), c->nk);
  hipLaunchKernelGGL(rows_to_c64_kernel, grid, dim3(256), 0, st, src, s_kstride, s_off, dst, d_kstride, d_off, cnt,
                     nvec, c->npwx, live);
  return check_launch(c, "to_c64", st);
}

pw_status launch_to_c128(pw_ctx* c, const cplx<float>* src, long s_kstride, const int* s_off, cplx<double>* dst,
                         long d_kstride, const int* d_off, const int* cnt, int nvec, hipStream_t st, const int* live) {
  dim3 grid(std::max(1, std::min(64, (nvec * c->npwx + 255) / 256)), c->nk);
  hipLaunchKernelGGL(rows_to_c128_kernel, grid, dim3(256), 0, st, src, s_kstride, s_off, dst, d_kstride, d_off,
                     cnt, nvec, c->npwx, live);
  return check_launch(c, "to_c128", st);
}

pw_status check_launch(pw_ctx* c, const char* what, hipStream_t st) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string(what) + " launch: " + hipGetErrorString(e));
  if (c->trace) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
  return PW_OK;
}

}  // namespace mkpw
