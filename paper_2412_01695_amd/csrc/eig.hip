// Batched small dense Hermitian kernels for the Rayleigh-Ritz step of the
// Davidson solver (Sec. 2.1, diagonalisation of the reduced N_base x N_base
// problem; Sec. 5.2 does it for many k-points at once on the GPU).
//
// heevx: the lowest nev eigenpairs of an n x n Hermitian matrix (n <= 64),
// one workgroup per k-point, everything in LDS:
//   1. Householder reduction to a Hermitian tridiagonal matrix,
//      Q^H A Q = T with Q = H_0 H_1 ... H_{n-3}, H_j = I - g_j u_j u_j^H
//      (Hermitian and unitary, g_j = 2 / |u_j|^2), each applied as the
//      rank-2 update A <- A - u w^H - w u^H with p = g A u,
//      w = p - (g/2)(u^H p) u; the u_j stay below the diagonal;
//   2. a diagonal phase change D (d_0 = 1, d_{j+1} = d_j e_j / |e_j|) making
//      T = D T_r D^H with T_r real symmetric, off-diagonal |e_j|;
//   3. eigenvalues of T_r by multisection on Sturm counts (8 points per step,
//      eight lanes per eigenvalue);
//   4. eigenvectors of T_r by inverse iteration, Gaussian elimination with
//      partial pivoting on T_r - lambda (one lane each, from a fixed
//      pseudo-random start, two solves: with lambda accurate to rounding each
//      solve shrinks the components along the other eigenvectors by their
//      gap over that error), then Gram-Schmidt (twice) within each cluster of
//      eigenvalues closer than 1e-3 of the matrix norm;
//   5. back through D and the reflectors: x = H_0 (... H_{n-3} (D y)), four
//      eigenvectors per wave at once.
// About (4/3) n^3 complex multiply-adds, against roughly 30 n^3 for the cyclic
// Jacobi sweeps this replaces.
//
// chol_inv: Cholesky S = L L^H of a small Hermitian positive-definite overlap
// and M = L^-H, used to orthonormalise a block of new basis vectors.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"
#include "wave.hpp"

namespace mkpw {

using cd = cplx<double>;

constexpr int kEigMax = 64;   // largest reduced problem
constexpr int kEigLd = kEigMax + 1;
// row stride of the real per-eigenpair arrays: in the inverse iteration lane t
// walks its own row, and the odd stride puts the lanes on different LDS banks
constexpr int kEigYs = kEigMax + 1;
constexpr int kEigNev = 32;   // most eigenpairs returned
constexpr int kEigThreads = 512;             // one workgroup per k-point
constexpr int kEigWaves = kEigThreads / 64;
constexpr int kEigPQ = 8;                    // work-items per row of the reduction (one DPP group)
static_assert(kEigPQ * kEigMax <= kEigThreads, "one row of the trailing block per group of kEigPQ");

// v on lane l of a wave, read into a wave-uniform value (l uniform)
__device__ __forceinline__ double lane_value(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// sum over the 64 lanes of a wave (every lane active), the same value on every
// lane: DPP sums within the rows of 16 lanes, then the four row sums read from
// lanes 0, 16, 32 and 48 (register reads, no LDS round trip)
__device__ __forceinline__ double wave_sum64(double v) {
  v += dpp<0xB1>(v);   // quad_perm 1,0,3,2
  v += dpp<0x4E>(v);   // quad_perm 2,3,0,1
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// 1/x for the reflectors and the inverse iteration: the hardware reciprocal
// estimate (relative error up to about 5e-8) refined by two Newton-Raphson
// steps r <- r + r (1 - x r) (each squares the relative error; measured to
// within rounding after the second), a few dependent operations instead of a
// full IEEE division
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}

// Householder reflector of a column held one component per lane, x_0 on lane
// h (h uniform), the rest on lanes h+1 .. mm-1, anything on the other lanes
// ignored: H = I - g u u^H with H x = beta e_0, beta = -e^{i arg x_0} |x|,
// u = x - beta e_0 (u on the same lanes as x); g = 0 (no reflection, beta =
// x_0) when x has nothing below its first component.  Called by a whole wave.
__device__ __forceinline__ void make_reflector(cd x, int h, int mm, int lane, double& g, cd& beta, cd& u) {
  const double sig = wave_sum64(lane > h && lane < mm ? x.x * x.x + x.y * x.y : 0.0);
  const double ar = lane_value(x.x, h), ai = lane_value(x.y, h);
  g = 0.0;
  beta = {ar, ai};
  u = x;
  if (sig > 0.0) {
    const double amag = sqrt(ar * ar + ai * ai);
    const double xn = sqrt(amag * amag + sig);
    const double xa = amag > 0.0 ? xn * rcp_nr(amag) : 0.0;
    beta = amag > 0.0 ? cd{-xa * ar, -xa * ai} : cd{-xn, 0.0};
    const cd u0 = {ar - beta.x, ai - beta.y};
    g = 2.0 * rcp_nr(u0.x * u0.x + u0.y * u0.y + sig);
    if (lane == h) u = u0;
  }
}

// The matrix is kept as its lower triangle, packed by rows (entry (i, j), i >=
// j, at i (i + 1) / 2 + j): the Hermitian reduction only updates the lower
// part of the trailing block and stores each reflector below the diagonal.
__device__ __forceinline__ int pk(int i, int j) { return (i * (i + 1) >> 1) + j; }
constexpr int kEigPacked = kEigMax * (kEigMax + 1) / 2;

// LDS: the packed matrix, then for nev eigenpairs the rows Y (eigenvectors of
// T_r) and U (two elimination rows per eigenpair), which the back-transformed
// eigenvectors Z (nev x kEigLd complex, fewer bytes) overwrite at the end,
// then the fixed part below.  At nev <= 24 the whole stays under 80 KiB, so
// two workgroups share a CU.
struct EigLds {
  cd ecx[kEigMax];                         // complex subdiagonal of T
  cd ph[kEigMax];                          // phases D
  cd pw[kEigMax];                          // p of the current reflector
  cd uu[2][kEigMax];                       // u of reflector j in uu[j & 1], by row of A
  double g[kEigMax];                       // reflector factors g_j
  double d[kEigMax], e[kEigMax];           // T_r
  double e2[kEigMax];                      // e_i^2 for the Sturm counts
  double lam[kEigNev];
  int cstart[kEigNev];                     // first index of each eigenvalue's cluster
  double scal[4];
};

__host__ __device__ constexpr size_t eig_region_bytes(int nev) {
  return ((size_t)3 * nev * kEigYs * sizeof(double) + 15) & ~(size_t)15;
}
__host__ __device__ constexpr size_t eig_lds_bytes(int nev) {
  return sizeof(cd) * kEigPacked + eig_region_bytes(nev) + sizeof(EigLds);
}

__global__ __launch_bounds__(kEigThreads) void heevx_kernel(const cd* __restrict__ Ag, long a_kstride, int lda,
                                                    const int* __restrict__ nk_arr, int nev_req,
                                                    double* __restrict__ w, cd* __restrict__ Vg, long v_kstride,
                                                    int ldv) {
  const int k = blockIdx.x;
  const int n = nk_arr[k];
  if (n <= 0) return;
  const int nev = min(nev_req, n);
  extern __shared__ __align__(16) unsigned char smem[];
  cd* A = reinterpret_cast<cd*>(smem);                         // packed lower triangle
  double* Yr = reinterpret_cast<double*>(A + kEigPacked);      // [nev][kEigYs]
  double* Ur = Yr + (size_t)nev_req * kEigYs;                  // [2 nev][kEigYs]
  cd* Zr = reinterpret_cast<cd*>(Yr);                          // [nev][kEigLd], at the end
  EigLds& S = *reinterpret_cast<EigLds*>(smem + sizeof(cd) * kEigPacked + eig_region_bytes(nev_req));
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const cd* Ak = Ag + (long)k * a_kstride;
  for (int e = tid; e < n * n; e += kEigThreads) {
    const int i = e / n, j = e - (e / n) * n;
    if (j > i) continue;
    const cd a = Ak[(long)i * lda + j], b = Ak[(long)j * lda + i];  // exact Hermitian part
    A[pk(i, j)] = {0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
  }
  __syncthreads();

  // ---- 1. Householder reduction, column j = 0 .. n-3 (trailing rows j+1 .. n-1).
  //         Two barriers per column: p = g A u over the trailing block, then the
  //         rank-2 update, during which wave 0 also updates column j+1 and
  //         forms its reflector from the new values held in registers.
  if (wave == 0 && n >= 3) {
    cd x = {0.0, 0.0};
    if (lane < n - 1) x = A[pk(1 + lane, 0)];
    double g0;
    cd beta, u;
    make_reflector(x, 0, n - 1, lane, g0, beta, u);
    if (lane < n - 1) {
      A[pk(1 + lane, 0)] = u;
      S.uu[0][1 + lane] = u;
    }
    if (lane == 0) {
      S.g[0] = g0;
      S.ecx[0] = beta;
    }
  }
  __syncthreads();
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;  // trailing size, 2 .. 63
    const double gj = S.g[j];  // uniform
    // row r of the trailing block on the eight work-items q of one lane group,
    // the last rows on wave 0, which forms the next reflector meanwhile and so
    // takes no rows of the update below once the block is 56 rows or fewer
    const int r = (kEigThreads / kEigPQ - 1) - (tid >> 3), q = tid & 7;
    const cd* uj = S.uu[j & 1];
    if (gj != 0.0) {
      // p_r = g sum_l A[j+1+r][j+1+l] u_l: each work-item takes l = q + 8 s,
      // in two batches of four whose loads are issued before their products
      cd acc = {0.0, 0.0};
      if (r < m) {
        const int i = j + 1 + r, ri = pk(i, 0);
#pragma unroll
        for (int h = 0; h < kEigMax / kEigPQ; h += 4) {
          if (q + kEigPQ * h >= m) break;  // nothing left in this row
          cd av[4], uv[4];
          // packed offset of row c, stepped along with c (no multiply per entry)
          int c = j + 1 + q + kEigPQ * h, rc = pk(c, 0);
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) {
            // A[i][c] from the lower triangle, conjugated above the diagonal;
            // past the block (c >= n) the diagonal entry, multiplied by u = 0
            av[s2] = A[c <= i ? ri + c : (c < n ? rc + i : ri + i)];
            uv[s2] = uj[c < n ? c : n - 1];
            rc += kEigPQ * c + kEigPQ * (kEigPQ + 1) / 2;
            c += kEigPQ;
          }
#pragma unroll
          for (int s2 = 0; s2 < 4; ++s2) {
            const int l = q + kEigPQ * (h + s2);
            const int c = j + 1 + l;
            const cd a = {av[s2].x, c <= i ? av[s2].y : -av[s2].y};
            const cd u = l < m ? uv[s2] : cd{0.0, 0.0};
            acc.x += a.x * u.x - a.y * u.y;
            acc.y += a.x * u.y + a.y * u.x;
          }
        }
      }
      // sum over the eight work-items of the row (DPP within groups of 8)
      acc.x += dpp<0xB1>(acc.x);
      acc.y += dpp<0xB1>(acc.y);
      acc.x += dpp<0x4E>(acc.x);
      acc.y += dpp<0x4E>(acc.y);
      acc.x += dpp<0x141>(acc.x);
      acc.y += dpp<0x141>(acc.y);
      if (r < m && q == 0) S.pw[r] = {gj * acc.x, gj * acc.y};
    }
    __syncthreads();
    // w = p - K u with K = (g/2) Re(u^H p), formed by every wave for itself
    double kk = 0.0;
    if (gj != 0.0) {
      cd p = {0.0, 0.0}, u = {0.0, 0.0};
      if (lane < m) {
        p = S.pw[lane];
        u = uj[j + 1 + lane];
      }
      kk = 0.5 * gj * wave_sum64(u.x * p.x + u.y * p.y);
    }
    if (wave == 0) {
      // column j+1 of the trailing block (row j+1+lane), updated in registers
      cd a = {0.0, 0.0};
      if (lane < m) a = A[pk(j + 1 + lane, j + 1)];
      if (gj != 0.0 && lane < m) {
        const cd ur = uj[j + 1 + lane], u0 = uj[j + 1];
        const cd pr = S.pw[lane], p0 = S.pw[0];
        const cd wr = {pr.x - kk * ur.x, pr.y - kk * ur.y}, w0 = {p0.x - kk * u0.x, p0.y - kk * u0.y};
        // a -= u_r conj(w_0) + w_r conj(u_0)
        a.x -= ur.x * w0.x + ur.y * w0.y + wr.x * u0.x + wr.y * u0.y;
        a.y -= ur.y * w0.x - ur.x * w0.y + wr.y * u0.x - wr.x * u0.y;
      }
      cd st = a;  // value stored at row j+1+lane of column j+1
      if (j + 3 < n) {
        // reflector of column j+1 from rows j+2 .. n-1, in place on lanes 1 .. m-1
        double g1;
        cd beta, u;
        make_reflector(a, 1, m, lane, g1, beta, u);
        if (lane >= 1) {
          st = u;
          if (lane < m) S.uu[(j + 1) & 1][j + 1 + lane] = u;
        }
        if (lane == 0) {
          S.g[j + 1] = g1;
          S.ecx[j + 1] = beta;
        }
      }
      if (lane < m) A[pk(j + 1 + lane, j + 1)] = st;
    }
    if (gj != 0.0 && r >= 1 && r < m) {
      // the rest of the trailing block (columns j+2 .., lower triangle):
      // A -= u w^H + w u^H; row r, columns l = 1 + q + 8 s <= r, in batches
      // of four whose loads are issued before their stores
      const cd ur = uj[j + 1 + r], pr = S.pw[r];
      const cd wr = {pr.x - kk * ur.x, pr.y - kk * ur.y};
#pragma unroll
      for (int h = 0; h < kEigMax / kEigPQ; h += 4) {
        if (1 + q + kEigPQ * h > r) break;  // nothing left in this row
        cd ul[4], pl[4], av[4];
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int l = 1 + q + kEigPQ * (h + s2), lc = l <= r ? l : 1;
          ul[s2] = uj[j + 1 + lc];
          pl[s2] = S.pw[lc];
          av[s2] = A[pk(j + 1 + r, j + 1 + lc)];
        }
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
          const int l = 1 + q + kEigPQ * (h + s2);
          if (l <= r) {
            const cd wl = {pl[s2].x - kk * ul[s2].x, pl[s2].y - kk * ul[s2].y};
            cd a = av[s2];
            // u_r conj(w_l) + w_r conj(u_l)
            a.x -= ur.x * wl.x + ur.y * wl.y + wr.x * ul[s2].x + wr.y * ul[s2].y;
            a.y -= ur.y * wl.x - ur.x * wl.y + wr.y * ul[s2].x - wr.x * ul[s2].y;
            A[pk(j + 1 + r, j + 1 + l)] = a;
          }
        }
      }
    }
    __syncthreads();
  }

  // ---- 2. T_r, the phases and the Gershgorin bounds, one lane per row
  //         (wave 0): the phases d_0 = 1, d_{i+1} = d_i e_i / |e_i| are a
  //         prefix product of unit numbers over the lanes
  if (wave == 0) {
    const int i = lane;
    double di = 0.0, mag = 0.0;
    cd u = {1.0, 0.0};
    if (i < n) di = A[pk(i, i)].x;
    if (i + 1 < n) {
      const cd ei = i == n - 2 ? A[pk(n - 1, n - 2)] : S.ecx[i];  // the last one has no reflector
      if (i == n - 2) S.ecx[i] = ei;
      mag = sqrt(ei.x * ei.x + ei.y * ei.y);
      if (mag > 0.0) u = {ei.x / mag, ei.y / mag};
    }
    cd p = u;  // inclusive product u_0 ... u_i
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const cd q = {__shfl_up(p.x, o, 64), __shfl_up(p.y, o, 64)};
      if (lane >= o) p = {q.x * p.x - q.y * p.y, q.x * p.y + q.y * p.x};
    }
    if (i < n) S.d[i] = di;
    if (i + 1 < n) {
      S.e[i] = mag;
      S.e2[i] = mag * mag;
      S.ph[i + 1] = p;
    }
    if (i == 0) S.ph[0] = {1.0, 0.0};
    const double eprev = __shfl_up(mag, 1, 64);
    const double r = (i > 0 ? eprev : 0.0) + mag;  // mag = 0 on the last row and beyond
    double lo = i < n ? di - r : 1e300, hi = i < n ? di + r : -1e300;
    double nrm = i < n ? fabs(di) + r : 0.0, emax2 = mag * mag;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      lo = fmin(lo, __shfl_xor(lo, o, 64));
      hi = fmax(hi, __shfl_xor(hi, o, 64));
      nrm = fmax(nrm, __shfl_xor(nrm, o, 64));
      emax2 = fmax(emax2, __shfl_xor(emax2, o, 64));
    }
    if (i == 0) {
      S.scal[0] = lo - 1e-14 * nrm - 1e-300;
      S.scal[1] = hi + 1e-14 * nrm + 1e-300;
      S.scal[2] = nrm;
      S.scal[3] = 2.3e-308 * fmax(1.0, emax2);  // smallest pivot allowed in the Sturm recurrence
    }
  }
  __syncthreads();

  // ---- 3. eigenvalues of T_r: eight work-items per eigenvalue, one point
  //         each; every step counts the eigenvalues below 8 interior points of
  //         the bracket (Sturm sequences) and keeps the ninth of it that holds
  //         eigenvalue t.  The stage is bound by the instructions one wave
  //         issues, so one sequence per work-item (more steps, each half as
  //         long) beats two, and more work-items per eigenvalue would put two
  //         waves on a SIMD.
  {
    const int t = tid >> 3, sub = tid & 7;
    if (t < nev) {  // whole groups of eight
      const double pivmin = S.scal[3];
      double lo = S.scal[0], hi = S.scal[1];
      for (int it = 0; it < 200; ++it) {
        if (!(hi - lo > 4.5e-16 * fmax(fabs(lo), fabs(hi)) + 1e-300)) break;
        const double xa = lo + (hi - lo) * ((sub + 1) / 9.0);
        int ca = 0;
        double qa = S.d[0] - xa;
        if (fabs(qa) < pivmin) qa = -pivmin;
        ca += qa < 0.0;
#pragma unroll 8
        for (int i = 1; i < n; ++i) {
          // 1/q from the hardware estimate and one Newton-Raphson step
          // (relative error about 2e-15): the count is that of T_r with its
          // e_i^2 perturbed at that level
          double rq = __builtin_amdgcn_rcp(qa);
          rq = fma(rq, fma(-qa, rq, 1.0), rq);
          qa = (S.d[i] - xa) - S.e2[i - 1] * rq;
          if (fabs(qa) < pivmin) qa = -pivmin;
          ca += qa < 0.0;
        }
        double lc = lo, hc = hi;
        if (ca <= t) lc = xa; else hc = xa;
        for (int o = 1; o < 8; o <<= 1) {
          lc = fmax(lc, __shfl_xor(lc, o, 64));
          hc = fmin(hc, __shfl_xor(hc, o, 64));
        }
        if (lc == lo && hc == hi) break;  // the points no longer split the bracket
        lo = lc;
        hi = hc;
      }
      if (sub == 0) S.lam[t] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();

  // ---- 4. eigenvectors of T_r, one lane per eigenpair (wave 0)
  if (wave == 0) {
    const double nrm = S.scal[2];
    const int t = lane;
    if (t < nev) {
      const double lm = S.lam[t];
      // inverse iteration on T_r - lm, rows kept in U[(2 t + c) * kEigYs + i];
      // the third elimination row is e_{i+1} where row i was pivoted (bit i
      // of `swapped`) and zero elsewhere, so it is not stored
      double* y = Yr + t * kEigYs;
      double* u0 = Ur + (2 * t + 0) * kEigYs;
      double* u1 = Ur + (2 * t + 1) * kEigYs;
      const double tiny = 2.2e-16 * fmax(nrm, 1e-300);
      unsigned h = 0x9E3779B9u * (unsigned)(t + 1);
      for (int i = 0; i < n; ++i) {  // fixed pseudo-random start in [-1, 1)
        h ^= h << 13;
        h ^= h >> 17;
        h ^= h << 5;
        y[i] = (double)(h & 0xFFFFFF) / 8388608.0 - 1.0;
      }
      for (int iter = 0; iter < 2; ++iter) {
        // forward elimination with partial pivoting, right-hand side y
        double c0 = S.d[0] - lm, c1 = n > 1 ? S.e[0] : 0.0, rc = y[0];
        unsigned long long swapped = 0;
#pragma unroll 4
        for (int i = 0; i + 1 < n; ++i) {
          const double s = S.e[i], dd = S.d[i + 1] - lm, ee = i + 2 < n ? S.e[i + 1] : 0.0, b1 = y[i + 1];
          // pivot row: the current one, or row i+1 (swapped: its third
          // entry ee is the implied u2); one reciprocal either way and no
          // divergent branch between the two cases
          const bool sw = !(fabs(c0) >= fabs(s));
          const double piv = sw ? s : c0, oth = sw ? c0 : s;
          const double l = piv != 0.0 ? oth * rcp_nr(piv) : 0.0;
          u0[i] = piv;
          u1[i] = sw ? dd : c1;
          y[i] = sw ? b1 : rc;
          if (sw) swapped |= 1ull << i;
          const double c0n = sw ? c1 - l * dd : dd - l * c1;
          c1 = sw ? -l * ee : ee;
          rc = sw ? rc - l * b1 : b1 - l * rc;
          c0 = c0n;
        }
        u0[n - 1] = c0;
        y[n - 1] = rc;
        // back substitution (tiny pivots replaced by eps |T|), then normalise
        double y1 = 0.0, y2 = 0.0, ss = 0.0;
#pragma unroll 4
        for (int i = n - 1; i >= 0; --i) {
          double piv = u0[i];
          if (fabs(piv) < tiny) piv = piv < 0.0 ? -tiny : tiny;
          const double u2i = i + 2 < n && ((swapped >> i) & 1ull) ? S.e[i + 1] : 0.0;
          const double v = (y[i] - (i + 1 < n ? u1[i] * y1 : 0.0) - (i + 2 < n ? u2i * y2 : 0.0)) * rcp_nr(piv);
          y[i] = v;
          y2 = y1;
          y1 = v;
          ss = fmax(ss, fabs(v));
        }
        const double sc = ss > 0.0 ? 1.0 / ss : 1.0;
        for (int i = 0; i < n; ++i) y[i] *= sc;
      }
    }
  }
  __syncthreads();
  // clusters of close eigenvalues (ascending)
  if (tid == 0) {
    int cs = 0;
    for (int i = 0; i < nev; ++i) {
      if (i > 0 && S.lam[i] - S.lam[i - 1] > 1e-3 * S.scal[2]) cs = i;
      S.cstart[i] = cs;
    }
  }
  __syncthreads();
  // Gram-Schmidt (twice) within each cluster, in ascending order; lane i owns
  // component i of every vector, so only the wave sums cross lanes
  if (wave == 0) {
    for (int t2 = 0; t2 < nev; ++t2) {
      double* yt = Yr + t2 * kEigYs;
      double v = lane < n ? yt[lane] : 0.0;
      for (int pass = 0; pass < 2; ++pass) {
        for (int s2 = S.cstart[t2]; s2 < t2; ++s2) {
          const double ys = lane < n ? Yr[s2 * kEigYs + lane] : 0.0;
          v -= wave_sum64(ys * v) * ys;
        }
        const double nn = wave_sum64(v * v);
        v *= nn > 0.0 ? 1.0 / sqrt(nn) : 0.0;
      }
      if (lane < n) yt[lane] = v;
    }
  }
  __syncthreads();

  // ---- 5. x = H_0 (... H_{n-3} (D y)): wave v takes eigenpairs v, v + 8, ...
  //         (at most four), all of them together so that their lane sums are
  //         independent and overlap; lane i holds component i
  {
    constexpr int kPerWave = kEigNev / kEigWaves;
    cd zi[kPerWave];
#pragma unroll
    for (int s2 = 0; s2 < kPerWave; ++s2) {
      const int t = wave + kEigWaves * s2;
      const double yv = (t < nev && lane < n) ? Yr[t * kEigYs + lane] : 0.0;
      zi[s2] = lane < n ? cd{S.ph[lane].x * yv, S.ph[lane].y * yv} : cd{0.0, 0.0};
    }
    __syncthreads();  // Z overwrites Y: every wave has its rows in registers first
    for (int j = n - 3; j >= 0; --j) {
      const double gj = S.g[j];
      if (gj == 0.0) continue;
      cd u = {0.0, 0.0};
      if (lane > j && lane < n) u = A[pk(lane, j)];
      double cr[kPerWave], ci[kPerWave];
#pragma unroll
      for (int s2 = 0; s2 < kPerWave; ++s2) {
        // c = g u^H z
        cr[s2] = wave_sum64(u.x * zi[s2].x + u.y * zi[s2].y);
        ci[s2] = wave_sum64(u.x * zi[s2].y - u.y * zi[s2].x);
      }
#pragma unroll
      for (int s2 = 0; s2 < kPerWave; ++s2) {
        const double a = gj * cr[s2], b = gj * ci[s2];
        zi[s2].x -= a * u.x - b * u.y;
        zi[s2].y -= a * u.y + b * u.x;
      }
    }
#pragma unroll
    for (int s2 = 0; s2 < kPerWave; ++s2) {
      const int t = wave + kEigWaves * s2;
      if (t < nev && lane < n) Zr[t * kEigLd + lane] = zi[s2];
    }
  }
  __syncthreads();
  if (tid < nev) w[(long)k * nev_req + tid] = S.lam[tid];
  cd* Vk = Vg + (long)k * v_kstride;
  for (int e = tid; e < n * nev; e += kEigThreads) {
    const int r = e / nev, t = e - (e / nev) * nev;
    Vk[(long)r * ldv + t] = Zr[t * kEigLd + r];
  }
}

constexpr int kCholMax = 32;

__global__ __launch_bounds__(64) void chol_inv_kernel(const cd* __restrict__ Sg, long s_kstride, int lds,
                                                      const int* __restrict__ nk_arr, cd* __restrict__ Mg,
                                                      long m_kstride, int ldm, int* __restrict__ info) {
  const int k = blockIdx.x;
  const int n = nk_arr[k];
  if (n <= 0) {
    if (threadIdx.x == 0) info[k] = 0;
    return;
  }
  __shared__ cd L[kCholMax][kCholMax + 1];
  __shared__ cd Li[kCholMax][kCholMax + 1];
  __shared__ int bad;
  __shared__ double dmax;
  const int tid = threadIdx.x;
  const cd* S = Sg + (long)k * s_kstride;
  for (int e = tid; e < n * n; e += 64) L[e / n][e % n] = S[(long)(e / n) * lds + (e % n)];
  if (tid == 0) {
    bad = 0;
    double m = 0.0;
    for (int i = 0; i < n; ++i) m = fmax(m, L[i][i].x);
    dmax = m;
  }
  __syncthreads();
  // right-looking: column j is final once the updates of the columns before it
  // are in; it is scaled, then the trailing lower triangle takes its rank-1
  // update, lane (row parity, column) = (tid / 32, tid % 32)
  const int cl = tid & 31, rp = tid >> 5;
  for (int j = 0; j < n; ++j) {
    const double d = L[j][j].x;
    if (tid == 0 && !(d > 1e-12 * dmax)) bad = 1;
    const double piv = sqrt(fmax(d, 1e-300)), inv = 1.0 / piv;
    for (int i = j + 1 + tid; i < n; i += 64) L[i][j] = {L[i][j].x * inv, L[i][j].y * inv};
    if (tid == 0) L[j][j] = {piv, 0.0};
    __syncthreads();
    const int c = j + 1 + cl;
    if (c < n) {
      const cd lc = L[c][j];
      for (int i = c + rp; i < n; i += 2) {  // L[i][c] -= L[i][j] conj(L[c][j])
        const cd a = L[i][j];
        L[i][c].x -= a.x * lc.x + a.y * lc.y;
        L[i][c].y -= a.y * lc.x - a.x * lc.y;
      }
    }
    __syncthreads();
  }
  // L^-1 row by row, right-looking: row q is final once the rows above have
  // been subtracted; it is scaled by 1/L_qq, then subtracted from the rows
  // below (Li starts as the identity; only c <= row is ever nonzero)
  for (int e = tid; e < n * kCholMax; e += 64) {
    const int i = e / kCholMax, cc = e - (e / kCholMax) * kCholMax;
    Li[i][cc] = {i == cc ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  for (int q = 0; q < n; ++q) {
    const double inv = 1.0 / L[q][q].x;
    if (tid <= q) Li[q][tid] = {Li[q][tid].x * inv, Li[q][tid].y * inv};
    __syncthreads();
    if (cl <= q) {
      const cd lq = Li[q][cl];
      for (int i = q + 1 + rp; i < n; i += 2) {  // Li[i][c] -= L[i][q] Li[q][c]
        const cd a = L[i][q];
        Li[i][cl].x -= a.x * lq.x - a.y * lq.y;
        Li[i][cl].y -= a.x * lq.y + a.y * lq.x;
      }
    }
    __syncthreads();
  }
  cd* M = Mg + (long)k * m_kstride;
  for (int e = tid; e < n * n; e += 64) {
    int i = e / n, j = e % n;  // M = Li^H (upper triangular)
    cd v = Li[j][i];
    M[(long)i * ldm + j] = {v.x, -v.y};
  }
  if (tid == 0) info[k] = bad;
}

pw_status launch_heev(pw_ctx* c, const cd* A, long a_kstride, int lda, const int* n, int nmax, int nev, double* w,
                      cd* V, long v_kstride, int ldv, hipStream_t st) {
  if (nmax > kEigMax) return set_err(c, PW_EINVAL, "reduced problem larger than 64");
  if (nev > kEigNev) return set_err(c, PW_EINVAL, "more than 32 eigenpairs requested");
  const size_t lds = eig_lds_bytes(nev);
  {
    pw_status s = ensure_lds_limit(c, (const void*)heevx_kernel, lds);
    if (s != PW_OK) return s;
  }
  hipLaunchKernelGGL(heevx_kernel, dim3(c->nk), dim3(kEigThreads), lds, st, A, a_kstride, lda, n, nev, w, V, v_kstride, ldv);
  return check_launch(c, "heevx", st);
}

pw_status launch_chol_inv(pw_ctx* c, const cd* S, long s_kstride, int lds, const int* n, cd* M, long m_kstride,
                          int ldm, int* info, hipStream_t st) {
  hipLaunchKernelGGL(chol_inv_kernel, dim3(c->nk), dim3(64), 0, st, S, s_kstride, lds, n, M, m_kstride, ldm, info);
  return check_launch(c, "chol_inv", st);
}

}  // namespace mkpw
