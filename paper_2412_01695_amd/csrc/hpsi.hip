// Batched H|psi> over many k-points: one fused kernel per precision and mesh.
//
// One workgroup applies H to one (k, band) row (Sec. 3, H application, all
// k-points and bands of the batch in one launch, Algorithm new_gpu):
//   1. scatter psi(G) into LDS "sticks" (one row per (m1', m2') that holds
//      plane waves) and, on the way, the projector overlaps
//      lambda_q = sum_G beta_q(k+G)^* psi(G) (Eq. lambdah), reduced over the
//      workgroup, and gamma = D lambda (Eq. gamma);
//   2. inverse 1D transforms along z on the sticks (Eq. zfft);
//   3. for a slab of z planes at a time: inverse along y (Eq. yfft) on the
//      occupied x columns, then along x (Eq. xfft) for every (y, z) line,
//      multiply by V(r)/N_r, forward along x, forward along y (Eq. fwFFT);
//   4. forward along z on the sticks;
//   5. gather back to the sphere and add the kinetic term (1/2)|k+G|^2 psi
//      and the nonlocal term sum_q gamma_q beta_q(k+G) (Eq. finalnl).
// Every 1D line is transformed in the registers of one work-item (fft.hpp);
// LDS carries the transposes between axes.  Nothing but psi, beta, the
// per-k maps and V(r) is read from memory and nothing but H psi is written:
// the paper's N_k x N_b full FFT meshes in global memory are never formed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "fft.hpp"
#include "internal.hpp"

namespace mkpw {

constexpr int kHpsiThreads = 256;
constexpr int kProjChunk = 8;

template <class T>
__device__ __forceinline__ cplx<T> ldc(const cplx<T>* p) {
  return *p;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// WC: compile-time capacity of the Miller window along each axis (>= the
// actual extents wx, wy, wz); entries beyond the actual window are zero.
template <class T, int N, int WC>
__global__ __launch_bounds__(kHpsiThreads) void hpsi_kernel(KTables t, VecSel sel, int nproj,
                                                           const cplx<T>* __restrict__ beta,
                                                           const cplx<T>* __restrict__ dij,
                                                           const T* __restrict__ vr,
                                                           const cplx<T>* __restrict__ psi,
                                                           cplx<T>* __restrict__ hpsi, int l3c, int ys,
                                                           int per_xcd, int ntask) {
  // XCD-aware order: consecutive (k, band) tasks run on the same XCD (blocks
  // are dealt to the 8 XCDs round-robin), so a k-point's projectors and maps
  // are fetched into one L2.
  const int bid = blockIdx.x;
  const int task = (bid & 7) * per_xcd + (bid >> 3);
  if (task >= ntask) return;
  const int ik = task / sel.nvec;
  const int iv = task - ik * sel.nvec;
  const int cnt = sel.cnt ? sel.cnt[ik] : sel.nvec;
  if (iv >= cnt) return;
  const int off = sel.off ? sel.off[ik] : 0;
  const int npwx = t.npwx;
  const long row = (long)ik * sel.kstride + (long)(off + iv) * npwx;
  const cplx<T>* __restrict__ p = psi + row;
  cplx<T>* __restrict__ hp = hpsi + row;
  const int npw = t.npw[ik];
  const int ns = t.nstick[ik];
  const int* __restrict__ gmap = t.gmap + (long)ik * npwx;
  const short* __restrict__ sof = t.sof + (long)ik * t.wx * t.wy;
  const double* __restrict__ kin = t.kin + (long)ik * npwx;
  const int wx = t.wx, wy = t.wy;
  constexpr int ZS = N | 1;  // stick row stride (odd: no LDS bank aliasing between sticks)

  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* Z = reinterpret_cast<cplx<T>*>(smem);  // [smax][ZS]
  cplx<T>* Y = Z + (size_t)t.smax * ZS;            // [l3c][N][ys], ys odd >= wx
  cplx<T>* red = Y + (size_t)l3c * N * ys;         // [4][kProjChunk]
  cplx<T>* gam = red + 4 * kProjChunk;             // [32]
  cplx<T>* lam = gam + 32;                         // [32]

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const cplx<T> zero = {T(0), T(0)};

  // ---- 1. zero the stick windows, scatter, projector overlaps
  for (int i = tid; i < ns * WC; i += kHpsiThreads) {
    int s = i / WC, j = i - s * WC;
    Z[s * ZS + j] = zero;
  }
  __syncthreads();
  for (int g = tid; g < npw; g += kHpsiThreads) {
    int gm = gmap[g];
    Z[(gm >> 8) * ZS + (gm & 255)] = p[g];
  }
  const cplx<T>* bk = beta + (long)ik * nproj * npwx;
  for (int q0 = 0; q0 < nproj; q0 += kProjChunk) {
    T ax[kProjChunk], ay[kProjChunk];
#pragma unroll
    for (int q = 0; q < kProjChunk; ++q) ax[q] = ay[q] = T(0);
    for (int g = tid; g < npw; g += kHpsiThreads) {
      cplx<T> v = p[g];
#pragma unroll
      for (int q = 0; q < kProjChunk; ++q) {
        if (q0 + q < nproj) {
          cplx<T> b = bk[(long)(q0 + q) * npwx + g];
          ax[q] += b.x * v.x + b.y * v.y;  // conj(b) * v
          ay[q] += b.x * v.y - b.y * v.x;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kProjChunk; ++q) {
      T sx = wave_sum(ax[q]), sy = wave_sum(ay[q]);
      if (lane == 0) red[wave * kProjChunk + q] = {sx, sy};
    }
    __syncthreads();
    if (tid < kProjChunk && q0 + tid < nproj) {
      cplx<T> s = red[tid];
      for (int w = 1; w < kHpsiThreads / 64; ++w) s = cadd(s, red[w * kProjChunk + tid]);
      lam[q0 + tid] = s;
    }
    __syncthreads();
  }
  if (tid < nproj) {
    cplx<T> s = zero;
    for (int q = 0; q < nproj; ++q) s = cadd(s, cmul(dij[tid * nproj + q], lam[q]));
    gam[tid] = s;
  }
  __syncthreads();

  // ---- 2. inverse z on the sticks: W inputs -> N outputs
  for (int s = tid; s < ns; s += kHpsiThreads) {
    cplx<T> v[N];
    sfor<N>([&](auto j) {
      constexpr int J = decltype(j)::value;
      if constexpr (J < WC) v[J] = Z[s * ZS + J];
      else v[J] = zero;
    });
    fft<T, N, +1>(v);
    sfor<N>([&](auto j) { Z[s * ZS + decltype(j)::value] = v[decltype(j)::value]; });
  }
  __syncthreads();

  // ---- 3. slabs of z planes.  V is stored permuted per slab so that the
  //         x-line work-items of a slab read it contiguously: Vp[slab][l1][lc][l2].
  for (int l30 = 0; l30 < N; l30 += l3c) {
    const int nl = min(l3c, N - l30);
    // inverse y on the occupied columns m1' < wx: W inputs (from the sticks) -> N outputs
    for (int i = tid; i < wx * nl; i += kHpsiThreads) {
      const int m1 = i % wx, lc = i / wx, l3 = l30 + lc;
      cplx<T> v[N];
      sfor<N>([&](auto j) {
        constexpr int J = decltype(j)::value;
        v[J] = zero;
        if constexpr (J < WC) {
          if (J < wy) {
            int s = sof[m1 * wy + J];
            if (s >= 0) v[J] = Z[s * ZS + l3];
          }
        }
      });
      fft<T, N, +1>(v);
      cplx<T>* y = Y + (size_t)lc * N * ys + m1;
      sfor<N>([&](auto l2) { y[decltype(l2)::value * ys] = v[decltype(l2)::value]; });
    }
    __syncthreads();
    // x lines: W inputs -> N points -> * V/N_r -> forward -> W outputs
    const T* vslab = vr + (size_t)l30 * N * N;
    for (int i = tid; i < N * nl; i += kHpsiThreads) {
      const int l2 = i % N, lc = i / N;
      cplx<T>* y = Y + ((size_t)lc * N + l2) * ys;
      cplx<T> v[N];
      sfor<N>([&](auto j) {
        constexpr int J = decltype(j)::value;
        if constexpr (J < WC) v[J] = (J < wx) ? y[J] : zero;
        else v[J] = zero;
      });
      fft<T, N, +1>(v);
      const T* vv = vslab + i;
      sfor<N>([&](auto l1) {
        constexpr int L1 = decltype(l1)::value;
        T f = vv[(size_t)L1 * nl * N];
        v[L1].x *= f;
        v[L1].y *= f;
      });
      fft<T, N, -1>(v);
      sfor<WC>([&](auto j) {
        constexpr int J = decltype(j)::value;
        if (J < wx) y[J] = v[J];
      });
    }
    __syncthreads();
    // forward y: N inputs -> W outputs, back into the sticks
    for (int i = tid; i < wx * nl; i += kHpsiThreads) {
      const int m1 = i % wx, lc = i / wx, l3 = l30 + lc;
      const cplx<T>* y = Y + (size_t)lc * N * ys + m1;
      cplx<T> v[N];
      sfor<N>([&](auto l2) { v[decltype(l2)::value] = y[decltype(l2)::value * ys]; });
      fft<T, N, -1>(v);
      sfor<WC>([&](auto j) {
        constexpr int J = decltype(j)::value;
        if (J < wy) {
          int s = sof[m1 * wy + J];
          if (s >= 0) Z[s * ZS + l3] = v[J];
        }
      });
    }
    __syncthreads();
  }

  // ---- 4. forward z on the sticks: N inputs -> W outputs
  for (int s = tid; s < ns; s += kHpsiThreads) {
    cplx<T> v[N];
    sfor<N>([&](auto j) { v[decltype(j)::value] = Z[s * ZS + decltype(j)::value]; });
    fft<T, N, -1>(v);
    sfor<WC>([&](auto j) { Z[s * ZS + decltype(j)::value] = v[decltype(j)::value]; });
  }
  __syncthreads();

  // ---- 5. gather + kinetic + nonlocal
  for (int g = tid; g < npwx; g += kHpsiThreads) {
    cplx<T> h = zero;
    if (g < npw) {
      int gm = gmap[g];
      h = Z[(gm >> 8) * ZS + (gm & 255)];
      cplx<T> v = p[g];
      T kk = (T)kin[g];
      h.x += kk * v.x;
      h.y += kk * v.y;
      for (int q = 0; q < nproj; ++q) h = cadd(h, cmul(bk[(long)q * npwx + g], gam[q]));
    }
    hp[g] = h;
  }
}

// ------------------------------------------------------------------ dispatch

namespace {

// V/N_r permuted for a slab width: Vp[l30 .. l30+nl)[l1][lc][l2] = V[l1][l2][l30+lc]
template <class T>
__global__ void permute_v_kernel(const T* __restrict__ v, T* __restrict__ vp, int n, int l3c) {
  const long nr = (long)n * n * n;
  for (long o = blockIdx.x * (long)blockDim.x + threadIdx.x; o < nr; o += (long)gridDim.x * blockDim.x) {
    const long slab_len = (long)l3c * n * n;
    const int l30 = (int)(o / slab_len) * l3c;
    const int nl = min(l3c, n - l30);
    long r = o - (long)l30 * n * n;
    const int l1 = (int)(r / ((long)nl * n));
    r -= (long)l1 * nl * n;
    const int lc = (int)(r / n), l2 = (int)(r % n);
    vp[o] = v[((long)l1 * n + l2) * n + l30 + lc];
  }
}

template <class T, int N, int WC>
pw_status launch_one(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st) {
  KTables t = c->tables();
  const size_t cs = sizeof(cplx<T>);
  const size_t zbytes = (size_t)t.smax * (N | 1) * cs;
  const size_t small = (4 * kProjChunk + 64) * cs;
  const int ys = t.wx | 1;
  const size_t plane = (size_t)N * ys * cs;
  // slab width: enough x lines to occupy the workgroup, within an LDS share
  // that leaves room for two workgroups per CU
  const size_t share = 80 * 1024;
  const size_t limit = 160 * 1024;
  long l3c = std::min<long>(N, std::max<long>(1, kHpsiThreads / N));
  while (l3c > 1 && zbytes + small + (size_t)l3c * plane > share) --l3c;
  size_t lds = zbytes + small + (size_t)l3c * plane;
  if (lds > limit) return set_err(c, PW_EINVAL, "H|psi> working set does not fit in LDS for this mesh");
  auto kern = hpsi_kernel<T, N, WC>;
  {
    pw_status s = ensure_lds_limit(c, (const void*)kern, lds);
    if (s != PW_OK) return s;
  }
  const long ntask = (long)t.nk * sel.nvec;
  if (ntask <= 0) return PW_OK;
  if (ntask > (1L << 30)) return set_err(c, PW_EINVAL, "too many (k, band) rows in one call");
  const bool fp64 = sizeof(T) == 8;
  // permuted potential for this slab width (built once per potential and width)
  int& have = fp64 ? c->vperm_l3c64 : c->vperm_l3c32;
  void*& vp = fp64 ? c->d_vperm64 : c->d_vperm32;
  if (have != (int)l3c || !vp) {
    if (!vp) {
      pw_status s = dev_alloc(c, (size_t)N * N * N * sizeof(T), &vp);
      if (s != PW_OK) return s;
    }
    const T* v = (const T*)(fp64 ? (const void*)c->d_v64 : (const void*)c->d_v32);
    hipLaunchKernelGGL(permute_v_kernel<T>, dim3(64), dim3(256), 0, st, v, (T*)vp, N, (int)l3c);
    have = (int)l3c;
  }
  const int per_xcd = (int)((ntask + 7) / 8);
  const unsigned nblk = 8u * (unsigned)per_xcd;
  const cplx<T>* beta = (const cplx<T>*)(fp64 ? c->d_beta64 : c->d_beta32);
  const cplx<T>* dij = (const cplx<T>*)(fp64 ? c->d_dij64 : c->d_dij32);
  hipLaunchKernelGGL(kern, dim3(nblk), dim3(kHpsiThreads), lds, st, t, sel, c->have_proj ? c->nproj : 0, beta,
                     dij, (const T*)vp, (const cplx<T>*)psi, (cplx<T>*)hpsi, (int)l3c, ys, per_xcd, (int)ntask);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string("h_psi launch: ") + hipGetErrorString(e));
  if (c->trace) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string("h_psi: ") + hipGetErrorString(e));
  }
  return PW_OK;
}

template <class T, int N>
pw_status launch_n(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st) {
  constexpr int kHalf = N / 2 + 2;
  const int w = std::max(c->wx, std::max(c->wy, c->wz));
  if (w <= kHalf) return launch_one<T, N, kHalf>(c, sel, psi, hpsi, st);
  return launch_one<T, N, N>(c, sel, psi, hpsi, st);
}

template <class T>
pw_status launch_t(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st) {
  switch (c->fft[0]) {
    case 15: return launch_n<T, 15>(c, sel, psi, hpsi, st);
    case 18: return launch_n<T, 18>(c, sel, psi, hpsi, st);
    case 20: return launch_n<T, 20>(c, sel, psi, hpsi, st);
    case 24: return launch_n<T, 24>(c, sel, psi, hpsi, st);
    case 30: return launch_n<T, 30>(c, sel, psi, hpsi, st);
    case 32: return launch_n<T, 32>(c, sel, psi, hpsi, st);
    case 36: return launch_n<T, 36>(c, sel, psi, hpsi, st);
    default: break;
  }
  return set_err(c, PW_EINVAL, "unsupported FFT mesh");
}

}  // namespace

bool hpsi_supported(int n1, int n2, int n3) {
  if (n1 != n2 || n1 != n3) return false;
  for (int n : {15, 18, 20, 24, 30, 32, 36})
    if (n == n1) return true;
  return false;
}

pw_status launch_hpsi(pw_ctx* c, pw_prec prec, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st) {
  if (!hpsi_supported(c->fft[0], c->fft[1], c->fft[2]))
    return set_err(c, PW_EINVAL,
                   "unsupported FFT mesh " + std::to_string(c->fft[0]) + "x" + std::to_string(c->fft[1]) + "x" +
                       std::to_string(c->fft[2]) + " (cubic 15, 18, 20, 24, 30, 32, 36)");
  if (prec == PW_FP64) return launch_t<double>(c, sel, psi, hpsi, st);
  return launch_t<float>(c, sel, psi, hpsi, st);
}

}  // namespace mkpw
