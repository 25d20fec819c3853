// Batched H|psi> over many k-points: one fused kernel per precision and mesh.
//
// One workgroup applies H to one (k, band) row (Sec. 3, H application, all
// k-points and bands of the batch in one launch, Algorithm new_gpu):
//   1. scatter psi(G) into LDS "sticks" (one row per (m1', m2') that holds
//      plane waves);
//   2. inverse 1D transforms along z on the sticks (Eq. zfft) -- and, on the
//      waves the sticks leave idle, the projector overlaps
//      lambda_q = sum_G beta_q(k+G)^* psi(G) (Eq. lambdah) and
//      gamma = D lambda (Eq. gamma);
//   3. for a slab of z planes at a time: inverse along y (Eq. yfft) on the
//      occupied x columns, then along x (Eq. xfft) for every (y, z) line,
//      multiply by V(r)/N_r, forward along x, forward along y (Eq. fwFFT);
//   4. forward along z on the sticks;
//   5. gather back to the sphere and add the kinetic term (1/2)|k+G|^2 psi
//      and the nonlocal term sum_q gamma_q beta_q(k+G) (Eq. finalnl).
// Each 1D line is transformed in registers (fft.hpp), by one work-item or by
// a pair of adjacent lanes; LDS carries the transposes between axes.  Nothing
// but psi, beta, the per-k maps and V(r) is read from memory and nothing but
// H psi is written: the paper's N_k x N_b full FFT meshes in global memory are
// never formed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fft.hpp"
#include "internal.hpp"

namespace mkpw {

constexpr int kHpsiThreads = 256;
constexpr int kProjChunk = 8;
constexpr int kMaxProj = 32;

// lane i takes lane i^1 (DPP quad permutation 1,0,3,2), i^2 (2,3,0,1), and the
// mirrors within 8 and 16 lanes
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// sum over the 64 lanes of a wavefront, returned on every lane: four DPP steps
// give each 16-lane row its sum, two lane shuffles combine the rows
template <class T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp<0xB1>(v);   // quad_perm 1,0,3,2
  v += dpp<0x4E>(v);   // quad_perm 2,3,0,1
  v += dpp<0x141>(v);  // row_half_mirror
  v += dpp<0x140>(v);  // row_mirror
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// The lane's half as a value the compiler cannot see through, so that the
// per-lane sign and twiddle selects stay next to their use instead of being
// hoisted out of the loops into long-lived registers.
__device__ __forceinline__ int lane_half(int h) {
  asm volatile("" : "+v"(h));
  return h;
}

// Per-row context.
template <class T>
struct Row {
  int ik, npw, ns, npwx;
  const cplx<T>* p;
  cplx<T>* hp;
  const int* gmap;
  const short* sof;
  const double* kin;
  const cplx<T>* bk;
};

// Decode the block into a (k, vector) row; false when the block has no row.
template <class T>
__device__ __forceinline__ bool row_of_block(const KTables& t, const VecSel& sel, int nproj, const cplx<T>* beta,
                                             const cplx<T>* psi, cplx<T>* hpsi, int per_xcd, int ntask, Row<T>& r) {
  // XCD-aware order: consecutive (k, band) tasks run on the same XCD (blocks
  // are dealt to the 8 XCDs round-robin), so a k-point's projectors and maps
  // are fetched into one L2.
  const int bid = blockIdx.x;
  const int task = (bid & 7) * per_xcd + (bid >> 3);
  if (task >= ntask) return false;
  const int ik = task / sel.nvec;
  const int iv = task - ik * sel.nvec;
  const int cnt = sel.cnt ? sel.cnt[ik] : sel.nvec;
  if (iv >= cnt) return false;
  const int off = sel.off ? sel.off[ik] : 0;
  r.ik = ik;
  r.npwx = t.npwx;
  const long row = (long)ik * sel.kstride + (long)(off + iv) * t.npwx;
  r.p = psi + row;
  r.hp = hpsi + row;
  r.npw = t.npw[ik];
  r.ns = t.nstick[ik];
  r.gmap = t.gmap + (long)ik * t.npwx;
  r.sof = t.sof + (long)ik * t.wx * t.wy;
  r.kin = t.kin + (long)ik * t.npwx;
  r.bk = beta + (long)ik * nproj * t.npwx;
  return true;
}

// Partial projector overlaps lambda_q = sum_G beta_q^* psi over the plane waves
// g = lt, lt + stride, ... of this work-item; each wave's sums go to red[wave][q].
template <class T>
__device__ __forceinline__ void project_partial(const Row<T>& r, int nproj, int lt, int stride, cplx<T>* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int q0 = 0; q0 < nproj; q0 += kProjChunk) {
    T ax[kProjChunk], ay[kProjChunk];
#pragma unroll
    for (int q = 0; q < kProjChunk; ++q) ax[q] = ay[q] = T(0);
    for (int g = lt; g < r.npw; g += stride) {
      cplx<T> v = r.p[g];
#pragma unroll
      for (int q = 0; q < kProjChunk; ++q) {
        if (q0 + q < nproj) {
          cplx<T> b = r.bk[(long)(q0 + q) * r.npwx + g];
          ax[q] += b.x * v.x + b.y * v.y;  // conj(b) * v
          ay[q] += b.x * v.y - b.y * v.x;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < kProjChunk; ++q) {
      if (q0 + q < nproj) {
        T sx = wave_sum(ax[q]), sy = wave_sum(ay[q]);
        if (lane == 0) red[wave * kMaxProj + q0 + q] = {sx, sy};
      }
    }
  }
}

// gamma_p = sum_q D_pq lambda_q with lambda_q summed over waves [w0, w1) of red
template <class T>
__device__ __forceinline__ void finish_gamma(int nproj, const cplx<T>* __restrict__ dij, const cplx<T>* red, int w0,
                                             int w1, cplx<T>* gam) {
  const int p = threadIdx.x;
  if (p >= nproj) return;
  cplx<T> g = {T(0), T(0)};
  for (int q = 0; q < nproj; ++q) {
    cplx<T> lam = {T(0), T(0)};
    for (int w = w0; w < w1; ++w) lam = cadd(lam, red[w * kMaxProj + q]);
    g = cadd(g, cmul(dij[p * nproj + q], lam));
  }
  gam[p] = g;
}

// Gather the local term from the sticks and add (1/2)|k+G|^2 psi and
// sum_q gamma_q beta_q (Eq. finalnl); the padding of the row is written as zero.
template <class T, int ZS>
__device__ __forceinline__ void gather_add(const Row<T>& r, int nproj, const cplx<T>* Z, const cplx<T>* gam) {
  const cplx<T> zero = {T(0), T(0)};
  for (int g = threadIdx.x; g < r.npwx; g += kHpsiThreads) {
    cplx<T> h = zero;
    if (g < r.npw) {
      int gm = r.gmap[g];
      h = Z[(gm >> 8) * ZS + (gm & 255)];
      cplx<T> v = r.p[g];
      T kk = (T)r.kin[g];
      h.x += kk * v.x;
      h.y += kk * v.y;
      for (int q = 0; q < nproj; ++q) h = cadd(h, cmul(r.bk[(long)q * r.npwx + g], gam[q]));
    }
    r.hp[g] = h;
  }
}

// ---------------------------------------------------------------- 1D passes
// Each pass comes in a one-work-item-per-line form and, for even N, a
// lane-pair form (pair_inverse / pair_forward in fft.hpp).

// inverse along one line: WC inputs from ld(m) -> N outputs to st(l, value)
template <class T, int N, int WC, bool PAIR, class LD, class ST>
__device__ __forceinline__ void line_inverse(int h, LD&& ld, ST&& st) {
  if constexpr (PAIR) {
    constexpr int M = N / 2;
    cplx<T> v[M];
    pair_inverse<T, N, WC, +1>(v, h, ld);
    sfor<M>([&](auto j) { st(2 * decltype(j)::value + h, v[decltype(j)::value]); });
  } else {
    cplx<T> v[N];
    sfor<N>([&](auto j) {
      constexpr int J = decltype(j)::value;
      if constexpr (J < WC) v[J] = ld(J);
      else v[J] = {T(0), T(0)};
    });
    fft<T, N, +1>(v);
    sfor<N>([&](auto j) { st(decltype(j)::value, v[decltype(j)::value]); });
  }
}

// forward along one line: N inputs from ld(l) -> the first WC outputs to st(m, value)
template <class T, int N, int WC, bool PAIR, class LD, class ST>
__device__ __forceinline__ void line_forward(int h, LD&& ld, ST&& st) {
  if constexpr (PAIR) {
    constexpr int M = N / 2;
    constexpr int KO = WC < M ? WC : M;
    cplx<T> v[M];
    sfor<M>([&](auto j) { v[decltype(j)::value] = ld(2 * decltype(j)::value + h); });
    pair_forward<T, N, WC, -1>(v, h);
    sfor<KO>([&](auto k) { st(decltype(k)::value + h * M, v[decltype(k)::value]); });
  } else {
    cplx<T> v[N];
    sfor<N>([&](auto j) { v[decltype(j)::value] = ld(decltype(j)::value); });
    fft<T, N, -1>(v);
    sfor<WC>([&](auto j) { st(decltype(j)::value, v[decltype(j)::value]); });
  }
}

// x line: WC inputs -> N points -> * V/N_r (vat(l1)) -> forward -> WC outputs
template <class T, int N, int WC, bool PAIR, class LD, class VAT, class ST>
__device__ __forceinline__ void line_xv(int h, LD&& ld, VAT&& vat, ST&& st) {
  if constexpr (PAIR) {
    constexpr int M = N / 2;
    constexpr int KO = WC < M ? WC : M;
    cplx<T> v[M];
    pair_inverse<T, N, WC, +1>(v, h, ld);
    sfor<M>([&](auto j) {
      constexpr int J = decltype(j)::value;
      T f = vat(2 * J + h);
      v[J].x *= f;
      v[J].y *= f;
    });
    pair_forward<T, N, WC, -1>(v, h);
    sfor<KO>([&](auto k) { st(decltype(k)::value + h * M, v[decltype(k)::value]); });
  } else {
    cplx<T> v[N];
    sfor<N>([&](auto j) {
      constexpr int J = decltype(j)::value;
      if constexpr (J < WC) v[J] = ld(J);
      else v[J] = {T(0), T(0)};
    });
    fft<T, N, +1>(v);
    sfor<N>([&](auto l) {
      constexpr int L = decltype(l)::value;
      T f = vat(L);
      v[L].x *= f;
      v[L].y *= f;
    });
    fft<T, N, -1>(v);
    sfor<WC>([&](auto j) { st(decltype(j)::value, v[decltype(j)::value]); });
  }
}

// ---------------------------------------------------------------- the kernel
// ZYP: z and y passes in lane pairs; XP: x pass in lane pairs (even N only).
// WC: compile-time capacity of the Miller window along each axis (>= the
// actual extents wx, wy, wz); entries beyond the actual window are zero.
template <class T, int N, int WC, bool ZYP, bool XP>
__global__ __launch_bounds__(kHpsiThreads) void hpsi_kernel(KTables t, VecSel sel, int nproj,
                                                           const cplx<T>* __restrict__ beta,
                                                           const cplx<T>* __restrict__ dij,
                                                           const T* __restrict__ vr,
                                                           const cplx<T>* __restrict__ psi,
                                                           cplx<T>* __restrict__ hpsi, int l3c, int ys,
                                                           int per_xcd, int ntask) {
  static_assert(!(ZYP || XP) || N % 2 == 0, "lane-pair passes need an even length");
  Row<T> r;
  if (!row_of_block(t, sel, nproj, beta, psi, hpsi, per_xcd, ntask, r)) return;
  const int wx = t.wx, wy = t.wy;
  const int ns = r.ns;
  constexpr int ZS = N | 1;  // stick row stride (odd: no LDS bank aliasing between sticks)

  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* Z = reinterpret_cast<cplx<T>*>(smem);   // [smax][ZS]
  cplx<T>* Y = Z + (size_t)t.smax * ZS;             // [l3c][N][ys], ys odd >= wx
  cplx<T>* red = Y + (size_t)l3c * N * ys;          // [4][kMaxProj]
  cplx<T>* gam = red + 4 * kMaxProj;                // [kMaxProj]
  short* sof = reinterpret_cast<short*>(gam + kMaxProj);  // [wx * wy] stick of (m1', m2')

  const int tid = threadIdx.x;
  const int h0 = tid & 1;
  const cplx<T> zero = {T(0), T(0)};
  constexpr int kZyStride = ZYP ? kHpsiThreads / 2 : kHpsiThreads;
  constexpr int kXStride = XP ? kHpsiThreads / 2 : kHpsiThreads;
  const int zy_slot = ZYP ? tid >> 1 : tid;
  const int x_slot = XP ? tid >> 1 : tid;

  // ---- 1. zero the stick windows, copy the stick map, scatter psi
  for (int i = tid; i < ns * WC; i += kHpsiThreads) {
    int s = i / WC, j = i - s * WC;
    Z[s * ZS + j] = zero;
  }
  for (int i = tid; i < wx * wy; i += kHpsiThreads) sof[i] = r.sof[i];
  __syncthreads();
  for (int g = tid; g < r.npw; g += kHpsiThreads) {
    int gm = r.gmap[g];
    Z[(gm >> 8) * ZS + (gm & 255)] = r.p[g];
  }
  __syncthreads();

  // ---- 2. inverse z on the sticks (W -> N) on the first waves; the projector
  //         overlaps on the waves the sticks leave idle
  const int zlanes = (ZYP ? 2 : 1) * ns;
  const int zwaves = min(kHpsiThreads / 64, (zlanes + 63) / 64);
  const bool proj_overlap = zwaves < kHpsiThreads / 64;
  if (tid < zwaves * 64) {
    for (int s = zy_slot; s < ns; s += (ZYP ? zwaves * 32 : zwaves * 64)) {
      const int h = lane_half(h0);
      cplx<T>* zr = Z + s * ZS;
      line_inverse<T, N, WC, ZYP>(h, [&](int m) { return zr[m]; }, [&](int l, cplx<T> v) { zr[l] = v; });
    }
  } else {
    project_partial(r, nproj, tid - zwaves * 64, kHpsiThreads - zwaves * 64, red);
  }
  __syncthreads();
  if (!proj_overlap) {
    project_partial(r, nproj, tid, kHpsiThreads, red);
    __syncthreads();
  }
  // gamma is first needed by the gather; the barriers of the slab loop publish it
  finish_gamma(nproj, dij, red, proj_overlap ? zwaves : 0, kHpsiThreads / 64, gam);

  // ---- 3. slabs of z planes.  V is stored permuted per slab so that the
  //         x-line work-items of a slab read it contiguously: Vp[slab][l1][lc][l2].
  for (int l30 = 0; l30 < N; l30 += l3c) {
    const int nl = min(l3c, N - l30);
    // inverse y on the occupied columns m1' < wx: W inputs (from the sticks) -> N outputs
    for (int i = zy_slot; i < wx * nl; i += kZyStride) {
      const int h = lane_half(h0);
      const int m1 = i % wx, lc = i / wx, l3 = l30 + lc;
      cplx<T>* y = Y + (size_t)lc * N * ys + m1;
      line_inverse<T, N, WC, ZYP>(
          h,
          [&](int m) {
            cplx<T> x = zero;
            if (m < wy) {
              int s = sof[m1 * wy + m];
              if (s >= 0) x = Z[s * ZS + l3];
            }
            return x;
          },
          [&](int l, cplx<T> v) { y[l * ys] = v; });
    }
    __syncthreads();
    // x lines: W inputs -> N points -> * V/N_r -> forward -> W outputs
    const T* vslab = vr + (size_t)l30 * N * N;
    for (int i = x_slot; i < N * nl; i += kXStride) {
      const int h = lane_half(h0);
      cplx<T>* y = Y + (size_t)i * ys;  // i = lc * N + l2
      const T* vv = vslab + i;
      line_xv<T, N, WC, XP>(
          h, [&](int m) { return m < wx ? y[m] : zero; }, [&](int l1) { return vv[(size_t)l1 * nl * N]; },
          [&](int m, cplx<T> v) {
            if (m < wx) y[m] = v;
          });
    }
    __syncthreads();
    // forward y: N inputs -> W outputs, back into the sticks
    for (int i = zy_slot; i < wx * nl; i += kZyStride) {
      const int h = lane_half(h0);
      const int m1 = i % wx, lc = i / wx, l3 = l30 + lc;
      const cplx<T>* y = Y + (size_t)lc * N * ys + m1;
      line_forward<T, N, WC, ZYP>(
          h, [&](int l) { return y[l * ys]; },
          [&](int m2, cplx<T> v) {
            if (m2 < wy) {
              int s = sof[m1 * wy + m2];
              if (s >= 0) Z[s * ZS + l3] = v;
            }
          });
    }
    __syncthreads();
  }

  // ---- 4. forward z on the sticks: N inputs -> W outputs (in place)
  for (int s = zy_slot; s < ns; s += kZyStride) {
    const int h = lane_half(h0);
    cplx<T>* zr = Z + s * ZS;
    line_forward<T, N, WC, ZYP>(
        h, [&](int l) { return zr[l]; },
        [&](int m3, cplx<T> v) {
          if (m3 < WC) zr[m3] = v;
        });
  }
  __syncthreads();

  // ---- 5. gather + kinetic + nonlocal
  gather_add<T, ZS>(r, nproj, Z, gam);
}

// V/N_r permuted for a slab width: Vp[l30 .. l30+nl)[l1][lc][l2] = V[l1][l2][l30+lc]
template <class T>
__global__ void permute_v_kernel(const T* __restrict__ v, T* __restrict__ vp, int n, int l3c) {
  const long nr = (long)n * n * n;
  for (long o = blockIdx.x * (long)blockDim.x + threadIdx.x; o < nr; o += (long)gridDim.x * blockDim.x) {
    const long slab_len = (long)l3c * n * n;
    const int l30 = (int)(o / slab_len) * l3c;
    const int nl = min(l3c, n - l30);
    long rr = o - (long)l30 * n * n;
    const int l1 = (int)(rr / ((long)nl * n));
    rr -= (long)l1 * nl * n;
    const int lc = (int)(rr / n), l2 = (int)(rr % n);
    vp[o] = v[((long)l1 * n + l2) * n + l30 + lc];
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

// Shape of one launch: kernel variant (1 = one work-item per line, 2 = lane
// pair per line, even N only) and slab width in z planes.
struct HpsiShape {
  int variant = 1;
  int l3c = 1;
};

template <class T, int N>
size_t hpsi_lds(const KTables& t, int l3c) {
  const size_t cs = sizeof(cplx<T>);
  return (size_t)t.smax * (N | 1) * cs + (5 * kMaxProj) * cs + (size_t)l3c * N * (t.wx | 1) * cs +
         ((size_t)t.wx * t.wy * sizeof(short) + 15) / 16 * 16;
}

template <class T, int N, int WC>
pw_status launch_shape(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st, HpsiShape sh) {
  KTables t = c->tables();
  const int ys = t.wx | 1;
  const int l3c = sh.l3c;
  const size_t lds = hpsi_lds<T, N>(t, l3c);
  auto kern = hpsi_kernel<T, N, WC, false, false>;
  if constexpr (N % 2 == 0) {
    if (sh.variant == 2) kern = hpsi_kernel<T, N, WC, true, true>;
    if (sh.variant == 3) kern = hpsi_kernel<T, N, WC, true, false>;
  }
  {
    pw_status s = ensure_lds_limit(c, (const void*)kern, lds);
    if (s != PW_OK) return s;
  }
  const long ntask = (long)t.nk * sel.nvec;
  if (ntask <= 0) return PW_OK;
  if (ntask > (1L << 30)) return set_err(c, PW_EINVAL, "too many (k, band) rows in one call");
  const bool fp64 = sizeof(T) == 8;
  // permuted potential for this slab width (rebuilt when the width changes)
  int& have = fp64 ? c->vperm_l3c64 : c->vperm_l3c32;
  void*& vp = fp64 ? c->d_vperm64 : c->d_vperm32;
  if (have != l3c || !vp) {
    if (!vp) {
      pw_status s = dev_alloc(c, (size_t)N * N * N * sizeof(T), &vp);
      if (s != PW_OK) return s;
    }
    const T* v = (const T*)(fp64 ? (const void*)c->d_v64 : (const void*)c->d_v32);
    hipLaunchKernelGGL(permute_v_kernel<T>, dim3(64), dim3(256), 0, st, v, (T*)vp, N, l3c);
    have = l3c;
  }
  const int per_xcd = (int)((ntask + 7) / 8);
  const unsigned nblk = 8u * (unsigned)per_xcd;
  const cplx<T>* beta = (const cplx<T>*)(fp64 ? c->d_beta64 : c->d_beta32);
  const cplx<T>* dij = (const cplx<T>*)(fp64 ? c->d_dij64 : c->d_dij32);
  hipLaunchKernelGGL(kern, dim3(nblk), dim3(kHpsiThreads), lds, st, t, sel, c->have_proj ? c->nproj : 0, beta,
                     dij, (const T*)vp, (const cplx<T>*)psi, (cplx<T>*)hpsi, l3c, ys, per_xcd, (int)ntask);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string("h_psi launch: ") + hipGetErrorString(e));
  if (c->trace) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string("h_psi: ") + hipGetErrorString(e));
  }
  return PW_OK;
}

// Candidate shapes: for each variant, the widest slab that fits in the LDS
// share for 1, 2 or 3 workgroups per CU, capped at the width that gives every
// work-item (or lane pair) one x line.
template <class T, int N>
std::vector<HpsiShape> hpsi_candidates(const KTables& t) {
  std::vector<HpsiShape> out;
  for (int variant : {1, 2, 3}) {
    if (variant != 1 && N % 2) continue;
    const int lanes = variant == 2 ? 2 : 1;  // work-items per x line
    const int cap = std::min(N, std::max(1, kHpsiThreads / (lanes * N)));
    for (size_t share : {size_t(53) * 1024, size_t(80) * 1024, size_t(160) * 1024}) {
      int l3c = std::min(N, share == 160 * 1024 ? N : cap);
      while (l3c > 1 && hpsi_lds<T, N>(t, l3c) > share) --l3c;
      if (hpsi_lds<T, N>(t, l3c) > 160 * 1024) continue;
      bool dup = false;
      for (auto& o : out) dup = dup || (o.variant == variant && o.l3c == l3c);
      if (!dup) out.push_back({variant, l3c});
    }
  }
  return out;
}

std::mutex g_tune_mu;
std::map<std::vector<long>, HpsiShape> g_tuned;

template <class T, int N, int WC>
pw_status launch_one(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st) {
  KTables t = c->tables();
  auto cands = hpsi_candidates<T, N>(t);
  if (cands.empty()) return set_err(c, PW_EINVAL, "H|psi> working set does not fit in LDS for this mesh");
  HpsiShape sh = cands[0];
  if (c->hpsi_variant != 0 || c->hpsi_slab != 0) {  // explicit shape
    if (c->hpsi_variant >= 2 && N % 2) return set_err(c, PW_EINVAL, "lane-pair variants need an even mesh");
    sh.variant = c->hpsi_variant ? (int)c->hpsi_variant : 1;
    sh.l3c = 0;
    for (auto& o : cands)
      if (o.variant == sh.variant) {
        sh.l3c = o.l3c;
        break;
      }
    if (c->hpsi_slab) sh.l3c = (int)std::min<int64_t>(c->hpsi_slab, N);
    if (sh.l3c < 1 || hpsi_lds<T, N>(t, sh.l3c) > 160 * 1024)
      return set_err(c, PW_EINVAL, "requested H|psi> slab does not fit in LDS");
    return launch_shape<T, N, WC>(c, sel, psi, hpsi, st, sh);
  }
  // autotune once per (precision, mesh, window, stick count, row-count bucket)
  long rows = 1;
  while (rows < (long)t.nk * sel.nvec) rows <<= 1;
  const std::vector<long> key = {(long)sizeof(T), N, WC, t.smax, t.wx, rows};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(key);
    if (it != g_tuned.end()) return launch_shape<T, N, WC>(c, sel, psi, hpsi, st, it->second);
  }
  if (cands.size() > 1) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(c, PW_EDEVICE, "hipEventCreate failed");
    }
    float best = 1e30f;
    for (auto& cand : cands) {
      pw_status s = launch_shape<T, N, WC>(c, sel, psi, hpsi, st, cand);  // warm-up (and V permutation)
      if (s != PW_OK) return s;
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < 2; ++r)
        if ((s = launch_shape<T, N, WC>(c, sel, psi, hpsi, st, cand)) != PW_OK) return s;
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms < best) {
        best = ms;
        sh = cand;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[key] = sh;
  }
  c->last_hpsi_variant = sh.variant;
  c->last_hpsi_slab = sh.l3c;
  return launch_shape<T, N, WC>(c, sel, psi, hpsi, st, sh);
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
