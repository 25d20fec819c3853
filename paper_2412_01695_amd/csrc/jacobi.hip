// Batched small dense Hermitian kernels for the Rayleigh-Ritz step of the
// Davidson solver (Sec. 2.1, diagonalisation of the reduced N_base x N_base
// problem; Sec. 5.2 does it for many k-points at once on the GPU).
//
// heev: cyclic Jacobi with the round-robin parallel ordering, one workgroup per
// k-point, matrix and eigenvectors in LDS.  Each rotation annihilates a_pq of
// the 2x2 block [[a, b], [b*, d]] (a, d real, b = |b| e^{i phi}) with
//   J = [[c, s e^{i phi}], [-s e^{-i phi}, c]],  A <- J^H A J,
// t = tan(theta) the smaller root of t^2 + 2 zeta t - 1 = 0,
// zeta = (d - a) / (2 |b|), c = 1/sqrt(1 + t^2), s = t c.
// Disjoint pairs commute, so a round applies all column rotations (A J, V J),
// then all row rotations (J^H A).  Sweeps stop when the off-diagonal
// Frobenius norm is below 1e-15 of the full norm.
//
// chol_inv: Cholesky S = L L^H of a small Hermitian positive-definite overlap
// and M = L^-H, used to orthonormalise a block of new basis vectors.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

namespace mkpw {

using cd = cplx<double>;

constexpr int kHeevMax = 64;
constexpr int kHeevLd = kHeevMax + 1;

__global__ __launch_bounds__(256) void heev_kernel(const cd* __restrict__ Ag, long a_kstride, int lda,
                                                   const int* __restrict__ nk_arr, int nev, double* __restrict__ w,
                                                   cd* __restrict__ Vg, long v_kstride, int ldv) {
  const int k = blockIdx.x;
  const int n = nk_arr[k];
  if (n <= 0) return;
  extern __shared__ __align__(16) unsigned char smem[];
  cd* A = reinterpret_cast<cd*>(smem);      // [n][kHeevLd]
  cd* V = A + kHeevMax * kHeevLd;           // [n][kHeevLd]
  __shared__ double rot[kHeevMax / 2][4];   // c, s, e^{i phi}
  __shared__ int pq[kHeevMax / 2][2];
  __shared__ double red[2][256];
  __shared__ int done;
  const int tid = threadIdx.x;
  const cd* Ak = Ag + (long)k * a_kstride;
  for (int e = tid; e < n * n; e += 256) {
    int i = e / n, j = e % n;
    cd a = Ak[(long)i * lda + j], b = Ak[(long)j * lda + i];  // exact Hermitian part
    A[i * kHeevLd + j] = {0.5 * (a.x + b.x), 0.5 * (a.y - b.y)};
    V[i * kHeevLd + j] = {i == j ? 1.0 : 0.0, 0.0};
  }
  __syncthreads();
  const int m = (n + 1) & ~1;  // even number of players; index n (if any) is a bye
  const int np = m / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    // convergence test on the off-diagonal norm
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += 256) {
      int i = e / n, j = e % n;
      cd a = A[i * kHeevLd + j];
      double v = a.x * a.x + a.y * a.y;
      tot += v;
      if (i != j) off += v;
    }
    red[0][tid] = off;
    red[1][tid] = tot;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
      if (tid < s) {
        red[0][tid] += red[0][tid + s];
        red[1][tid] += red[1][tid + s];
      }
      __syncthreads();
    }
    if (tid == 0) done = (red[0][0] <= 1e-30 * red[1][0]) || red[0][0] == 0.0;
    __syncthreads();
    if (done) break;
    for (int r = 0; r < m - 1; ++r) {
      if (tid < np) {
        int a, b;
        if (tid == 0) {
          a = m - 1;
          b = r;
        } else {
          a = (r + tid) % (m - 1);
          b = (r - tid + m - 1) % (m - 1);
        }
        int p = min(a, b), q = max(a, b);
        double c = 1.0, s = 0.0, er = 1.0, ei = 0.0;
        if (q < n) {
          cd apq = A[p * kHeevLd + q];
          double mag = sqrt(apq.x * apq.x + apq.y * apq.y);
          double app = A[p * kHeevLd + p].x, aqq = A[q * kHeevLd + q].x;
          if (mag > 1e-300 && mag > 1e-18 * (fabs(app) + fabs(aqq))) {
            double zeta = (aqq - app) / (2.0 * mag);
            double t = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
            c = 1.0 / sqrt(1.0 + t * t);
            s = t * c;
            er = apq.x / mag;
            ei = apq.y / mag;
          }
        }
        pq[tid][0] = p;
        pq[tid][1] = q;
        rot[tid][0] = c;
        rot[tid][1] = s;
        rot[tid][2] = er;
        rot[tid][3] = ei;
      }
      __syncthreads();
      // columns: A <- A J, V <- V J
      for (int e = tid; e < np * n; e += 256) {
        int t = e / n, i = e % n;
        int p = pq[t][0], q = pq[t][1];
        double s = rot[t][1];
        if (q >= n || s == 0.0) continue;
        double c = rot[t][0], er = rot[t][2], ei = rot[t][3];
        // col p' = c x - s e^{-i phi} y ; col q' = s e^{i phi} x + c y
        cd x = A[i * kHeevLd + p], y = A[i * kHeevLd + q];
        A[i * kHeevLd + p] = {c * x.x - s * (er * y.x + ei * y.y), c * x.y - s * (er * y.y - ei * y.x)};
        A[i * kHeevLd + q] = {s * (er * x.x - ei * x.y) + c * y.x, s * (er * x.y + ei * x.x) + c * y.y};
        x = V[i * kHeevLd + p];
        y = V[i * kHeevLd + q];
        V[i * kHeevLd + p] = {c * x.x - s * (er * y.x + ei * y.y), c * x.y - s * (er * y.y - ei * y.x)};
        V[i * kHeevLd + q] = {s * (er * x.x - ei * x.y) + c * y.x, s * (er * x.y + ei * x.x) + c * y.y};
      }
      __syncthreads();
      // rows: A <- J^H A ; row p' = c x - s e^{i phi} y ; row q' = s e^{-i phi} x + c y
      for (int e = tid; e < np * n; e += 256) {
        int t = e / n, j = e % n;
        int p = pq[t][0], q = pq[t][1];
        double s = rot[t][1];
        if (q >= n || s == 0.0) continue;
        double c = rot[t][0], er = rot[t][2], ei = rot[t][3];
        cd x = A[p * kHeevLd + j], y = A[q * kHeevLd + j];
        A[p * kHeevLd + j] = {c * x.x - s * (er * y.x - ei * y.y), c * x.y - s * (er * y.y + ei * y.x)};
        A[q * kHeevLd + j] = {s * (er * x.x + ei * x.y) + c * y.x, s * (er * x.y - ei * x.x) + c * y.y};
      }
      __syncthreads();
    }
  }
  // lowest nev eigenpairs in ascending order (ties keep the index order)
  for (int i = tid; i < n; i += 256) {
    double li = A[i * kHeevLd + i].x;
    int rank = 0;
    for (int j = 0; j < n; ++j) {
      double lj = A[j * kHeevLd + j].x;
      rank += (lj < li) || (lj == li && j < i);
    }
    if (rank < nev) {
      w[(long)k * nev + rank] = li;
      cd* Vk = Vg + (long)k * v_kstride;
      for (int r = 0; r < n; ++r) Vk[(long)r * ldv + rank] = V[r * kHeevLd + i];
    }
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
  for (int j = 0; j < n; ++j) {
    if (tid == 0) {
      double d = L[j][j].x;
      for (int q = 0; q < j; ++q) d -= L[j][q].x * L[j][q].x + L[j][q].y * L[j][q].y;
      if (!(d > 1e-12 * dmax)) bad = 1;
      L[j][j] = {sqrt(fmax(d, 1e-300)), 0.0};
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < n; i += 64) {
      double xr = L[i][j].x, xi = L[i][j].y;
      for (int q = 0; q < j; ++q) {  // - L[i][q] conj(L[j][q])
        cd a = L[i][q], b = L[j][q];
        xr -= a.x * b.x + a.y * b.y;
        xi -= a.y * b.x - a.x * b.y;
      }
      double inv = 1.0 / L[j][j].x;
      L[i][j] = {xr * inv, xi * inv};
    }
    __syncthreads();
  }
  // columns of L^-1 by forward substitution, one column per work-item
  for (int c = tid; c < n; c += 64) {
    for (int i = 0; i < n; ++i) Li[i][c] = {0.0, 0.0};
    for (int i = c; i < n; ++i) {
      double xr = (i == c) ? 1.0 : 0.0, xi = 0.0;
      for (int q = c; q < i; ++q) {
        cd a = L[i][q], b = Li[q][c];
        xr -= a.x * b.x - a.y * b.y;
        xi -= a.x * b.y + a.y * b.x;
      }
      double inv = 1.0 / L[i][i].x;
      Li[i][c] = {xr * inv, xi * inv};
    }
  }
  __syncthreads();
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
  if (nmax > kHeevMax) return set_err(c, PW_EINVAL, "reduced problem larger than 64");
  const size_t lds = 2 * (size_t)kHeevMax * kHeevLd * sizeof(cd);
  {
    pw_status s = ensure_lds_limit(c, (const void*)heev_kernel, lds);
    if (s != PW_OK) return s;
  }
  hipLaunchKernelGGL(heev_kernel, dim3(c->nk), dim3(256), lds, st, A, a_kstride, lda, n, nev, w, V, v_kstride, ldv);
  return check_launch(c, "heev", st);
}

pw_status launch_chol_inv(pw_ctx* c, const cd* S, long s_kstride, int lds, const int* n, cd* M, long m_kstride,
                          int ldm, int* info, hipStream_t st) {
  hipLaunchKernelGGL(chol_inv_kernel, dim3(c->nk), dim3(64), 0, st, S, s_kstride, lds, n, M, m_kstride, ldm, info);
  return check_launch(c, "chol_inv", st);
}

}  // namespace mkpw
