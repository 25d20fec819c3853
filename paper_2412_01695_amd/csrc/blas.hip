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

// ------------------------------------------------------------------ gram on the FP64 matrix cores

// D (16 x 16) += A (16 x 4) B (4 x 16) per wave: lane l holds A[l % 16][l / 16]
// and B[l / 16][l % 16]; item r of the result is D[4 r + l / 16][l % 16]
typedef double mf64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mf64x4 mfma4(double a, double b, mf64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kMB = 32;  // C block per workgroup (4 waves, one 16 x 16 tile each)
constexpr int kMK = 32;  // plane waves per chunk staged in LDS

// C = alpha A^H B per k (rows i < a_cnt of A, j < b_cnt of B, inner products
// over the k's npw plane waves), written at (c_roff + i, c_coff + j), with the
// products on the matrix cores: the
// workgroup stages 32 rows of A and of B, 32 plane waves at a time, with
// coalesced loads into LDS (rows padded by one element against bank
// conflicts), and each wave forms a 16 x 16 tile, four plane waves per step
// (four real products per complex step: Re = ar br + ai bi, Im = ar bi - ai br).
__global__ __launch_bounds__(256) void gram_mfma_kernel(GramArgs a) {
  const int k = blockIdx.x;
  const int ni = sel_i(a.a_cnt, k, a.a_n);
  const int nj = sel_i(a.b_cnt, k, a.b_n);
  const int i0 = blockIdx.y * kMB, j0 = blockIdx.z * kMB;
  if (i0 >= ni || j0 >= nj) return;
  if (a.b_live) {  // a block none of whose B vectors takes part is skipped
    const int* lv = a.b_live + (long)k * a.live_kstride;
    bool any = false;
    for (int j = j0; j < min(j0 + kMB, nj); ++j) any |= lv[j] != 0;
    if (!any) return;
  }
  const int npw = a.npw[k];
  const c64d* A = a.A + (long)k * a.a_kstride + (long)sel_i(a.a_off, k, a.a_row) * a.ld;
  const c64d* B = a.B + (long)k * a.b_kstride + (long)sel_i(a.b_off, k, a.b_row) * a.ld;
  __shared__ c64d As[kMB][kMK + 1];
  __shared__ c64d Bs[kMB][kMK + 1];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ti = wave >> 1, tj = wave & 1;  // this wave's tile of the block
  const int l16 = lane & 15, kq = lane >> 4;
  // a wave whose tile lies wholly past ni or nj (small blocks) stages its
  // share of the chunk but forms no products
  const bool live = i0 + 16 * ti < ni && j0 + 16 * tj < nj;
  mf64x4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
  // the next chunk's loads are issued into registers before this chunk's
  // products, so their latency is hidden behind the matrix cores
  constexpr int kQ = kMB * kMK / 256;
  c64d pa[kQ], pb[kQ];
  auto fetch = [&](int g0) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = tid + q * 256, r = e / kMK, g = e % kMK;
      const bool gok = g0 + g < npw;
      pa[q] = gok && i0 + r < ni ? A[(long)(i0 + r) * a.ld + g0 + g] : c64d{0.0, 0.0};
      pb[q] = gok && j0 + r < nj ? B[(long)(j0 + r) * a.ld + g0 + g] : c64d{0.0, 0.0};
    }
  };
  fetch(0);
  for (int g0 = 0; g0 < npw; g0 += kMK) {
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int e = tid + q * 256, r = e / kMK, g = e % kMK;
      As[r][g] = pa[q];
      Bs[r][g] = pb[q];
    }
    __syncthreads();
    if (g0 + kMK < npw) fetch(g0 + kMK);
#pragma unroll
    for (int kk = 0; kk < kMK && live; kk += 4) {
      const c64d x = As[16 * ti + l16][kk + kq], y = Bs[16 * tj + l16][kk + kq];
      cr = mfma4(x.x, y.x, cr);
      cr = mfma4(x.y, y.y, cr);
      ci = mfma4(x.x, y.y, ci);
      ci = mfma4(-x.y, y.x, ci);
    }
    __syncthreads();
  }
  c64d* C = a.C + (long)k * a.c_kstride;
  const int r0 = sel_i(a.c_roff, k, a.c_row), c0 = sel_i(a.c_coff, k, a.c_col);
  const int j = j0 + 16 * tj + l16;
  if (j >= nj || (a.b_live && !a.b_live[(long)k * a.live_kstride + j])) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = i0 + 16 * ti + 4 * r + kq;
    if (i >= ni) continue;
    const int row = r0 + i, col = c0 + j;
    const double vr = a.alpha * cr[r], vi = a.alpha * ci[r];
    C[(long)row * a.ldc + col] = {vr, vi};
    // mirrored entry, unless that position is itself computed directly
    if (a.mirror && !(col >= r0 && col < r0 + ni && row >= c0 && row < c0 + nj)) C[(long)col * a.ldc + row] = {vr, -vi};
  }
}

// ------------------------------------------------------------------ rows_combine on the FP64 matrix cores

// Y_j = [Y_j +] alpha sum_i X_i C(c_roff + i, c_coff + j) per k, for j <
// y_cnt, i < x_cnt (at most 64), over all npwx entries of a row, with the
// products on the matrix cores: a workgroup covers 64 plane waves (16 per
// wave) and every output row; for each block of 16 output rows the C entries
// (ni x 16) are staged in LDS, and a wave forms its 16 x 16 tile (output rows
// x plane waves) four input rows per step, the X entries loaded straight from
// memory (16 consecutive plane waves of 4 rows per load).
__global__ __launch_bounds__(256) void rows_combine_mfma_kernel(CombArgs a) {
  const int k = blockIdx.y;
  const int ni = sel_i(a.x_cnt, k, a.x_n);
  const int nj = sel_i(a.y_cnt, k, a.y_n);
  if (nj <= 0) return;
  const int npwx = a.ld;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int l16 = lane & 15, kq = lane >> 4;
  const int g = blockIdx.x * 64 + wave * 16 + l16;  // this lane's B column (plane wave)
  const bool gok = g < npwx;
  const c64d* X = a.X + (long)k * a.x_kstride + (long)sel_i(a.x_off, k, a.x_row) * npwx;
  c64d* Y = a.Y + (long)k * a.y_kstride + (long)sel_i(a.y_off, k, a.y_row) * npwx;
  const c64d* Cm = a.Cm + (long)k * a.c_kstride + (long)sel_i(a.c_roff, k, a.c_row) * a.ldc +
                   sel_i(a.c_coff, k, a.c_col);
  const int* lv = a.y_live ? a.y_live + (long)k * a.live_kstride : nullptr;
  __shared__ c64d cs[64][17];  // C(i, j0 + jj), padded
  for (int j0 = 0; j0 < nj; j0 += 16) {
    if (lv) {  // a block none of whose output rows takes part is skipped (uniform over the block)
      bool any = false;
      for (int jj = j0; jj < min(j0 + 16, nj); ++jj) any |= lv[jj] != 0;
      if (!any) continue;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 16; e += 256) {
      const int i = e / 16, jj = e % 16;
      cs[i][jj] = i < ni && j0 + jj < nj ? Cm[(long)i * a.ldc + j0 + jj] : c64d{0.0, 0.0};
    }
    __syncthreads();
    mf64x4 dr = {0.0, 0.0, 0.0, 0.0}, di = {0.0, 0.0, 0.0, 0.0};
    // four steps of four input rows at a time, their X loads issued first
    // (rows past ni read row 0 and meet a zero C entry)
    for (int i0 = 0; i0 < ni; i0 += 16) {
      c64d xs[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int i = i0 + 4 * u + kq;
        xs[u] = gok ? X[(long)(i < ni ? i : 0) * npwx + g] : c64d{0.0, 0.0};
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (i0 + 4 * u >= ni) break;
        // A = C^T (row: output j = l16, column: input i); B = X (row i, column g)
        const c64d c = cs[i0 + 4 * u + kq][l16];
        dr = mfma4(c.x, xs[u].x, dr);
        dr = mfma4(-c.y, xs[u].y, dr);
        di = mfma4(c.x, xs[u].y, di);
        di = mfma4(c.y, xs[u].x, di);
      }
    }
    if (!gok) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = j0 + 4 * r + kq;
      if (j >= nj || (lv && !lv[j])) continue;
      c64d* y = Y + (long)j * npwx + g;
      const c64d o = a.accumulate ? *y : c64d{0.0, 0.0};
      *y = {o.x + a.alpha * dr[r], o.y + a.alpha * di[r]};
    }
  }
}

// ------------------------------------------------------------------ in-place Y <- Y M, M upper triangular

// n <= NB rows of Y per k (NB a multiple of 8, at most 32): a work-item owns
// one column g of the rows; row i is read once and added into the outputs
// j >= i it feeds (Y_j = sum_{i <= j} Y_i M_ij, outputs in registers), both
// loops unrolled so that only the triangle is formed; every row is read
// before the first is written
template <int NB>
__global__ __launch_bounds__(256) void rows_trmm_kernel(c64d* Yb, long y_kstride, const int* y_off, const int* y_cnt,
                                                        int npwx, const c64d* Mb, long m_kstride, int ldm) {
  const int k = blockIdx.y;
  const int n = y_cnt[k];
  if (n <= 0) return;
  const int g = blockIdx.x * 256 + threadIdx.x;
  c64d* Y = Yb + (long)k * y_kstride + (long)y_off[k] * npwx;
  const c64d* M = Mb + (long)k * m_kstride;
  __shared__ c64d ms[NB * NB];
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int i = e / NB, j = e - (e / NB) * NB;
    ms[e] = i < n && j < n ? M[(long)i * ldm + j] : c64d{0.0, 0.0};
  }
  __syncthreads();
  if (g >= npwx) return;
  double ar[NB], ai[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) ar[j] = ai[j] = 0.0;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    if (i < n) {
      const c64d x = Y[(long)i * npwx + g];
#pragma unroll
      for (int j = i; j < NB; ++j) {
        const c64d c = ms[i * NB + j];
        ar[j] += x.x * c.x - x.y * c.y;
        ai[j] += x.x * c.y + x.y * c.x;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NB; ++j)
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
  dim3 grid(c->nk, (ni_max + kMB - 1) / kMB, (nj_max + kMB - 1) / kMB);
  hipLaunchKernelGGL(gram_mfma_kernel, grid, dim3(256), 0, st, a);
  return check_launch(c, "gram", st);
}

pw_status launch_combine(pw_ctx* c, const CombArgs& a, int ni_max, hipStream_t st) {
  if (ni_max > 64) return set_err(c, PW_EINVAL, "rows_combine: more than 64 input rows");
  dim3 grid((a.ld + 63) / 64, c->nk);
  hipLaunchKernelGGL(rows_combine_mfma_kernel, grid, dim3(256), 0, st, a);
  return check_launch(c, "rows_combine", st);
}

pw_status launch_trmm(pw_ctx* c, cplx<double>* Y, long y_kstride, const int* y_off, const int* y_cnt,
                      const cplx<double>* M, long m_kstride, int ldm, hipStream_t st) {
  // the row counts y_cnt are at most ldm (the order of M)
  if (ldm < 1 || ldm > 32) return set_err(c, PW_EINVAL, "triangular factor larger than 32");
  dim3 grid((c->npwx + 255) / 256, c->nk);
#define MKPW_TRMM(NB)                                                                                          \
  hipLaunchKernelGGL(rows_trmm_kernel<NB>, grid, dim3(256), 0, st, Y, y_kstride, y_off, y_cnt, c->npwx, M, m_kstride, \
                     ldm)
  switch ((ldm + 7) / 8) {
    case 1: MKPW_TRMM(8); break;
    case 2: MKPW_TRMM(16); break;
    case 3: MKPW_TRMM(24); break;
    default: MKPW_TRMM(32); break;
  }
#undef MKPW_TRMM
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
