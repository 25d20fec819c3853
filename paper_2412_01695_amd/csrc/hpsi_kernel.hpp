// Batched H|psi> over many k-points: the fused kernel and its launch machinery,
// instantiated per mesh size in hpsi_n<N>.hip.
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
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fft.hpp"
#include "internal.hpp"
#include "wave.hpp"

namespace mkpw {
constexpr int kProjChunk = 8;
constexpr int kMaxProj = 32;

// The lane's half as a value the compiler cannot see through, so that the
// per-lane sign and twiddle selects stay next to their use instead of being
// hoisted out of the loops into long-lived registers.
__device__ __forceinline__ int lane_half(int h) {
  asm volatile("" : "+v"(h));
  return h;
}

// LDS pointers carry their address space, so that index arithmetic on them
// is 32-bit; complex values are moved through them member by member.
template <class U>
using lds_t = __attribute__((address_space(3))) U;
template <class T>
__device__ __forceinline__ cplx<T> lds_ld(const lds_t<cplx<T>>* p) {
  return {p->x, p->y};
}
template <class T>
__device__ __forceinline__ void lds_st(lds_t<cplx<T>>* p, cplx<T> v) {
  p->x = v.x;
  p->y = v.y;
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
  if (sel.live && !sel.live[task]) return false;
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

// gamma_p = sum_q D_pq lambda_q (Eq. gamma), lambda_q summed over the nslot
// per-wave partial sums in red[w][q]; D is staged in LDS (dl[p][q]).
template <class T>
__device__ __forceinline__ void finish_gamma(int p, int nproj, const lds_t<cplx<T>>* dl, const lds_t<cplx<T>>* red,
                                             int nslot, lds_t<cplx<T>>* gam) {
  cplx<T> g = {T(0), T(0)};
  for (int q = 0; q < nproj; ++q) {
    cplx<T> lam = {T(0), T(0)};
    for (int w = 0; w < nslot; ++w) lam = cadd(lam, lds_ld(red + w * nproj + q));
    g = cadd(g, cmul(lds_ld(dl + p * nproj + q), lam));
  }
  lds_st(gam + p, g);
}

// Gather the local term from the sticks and add (1/2)|k+G|^2 psi and
// sum_q gamma_q beta_q (Eq. finalnl); the padding of the row is written as zero.
template <class T, int ZS, int NT>
__device__ __forceinline__ void gather_add(const Row<T>& r, int nproj, const lds_t<cplx<T>>* Z,
                                           const lds_t<cplx<T>>* gam) {
  const cplx<T> zero = {T(0), T(0)};
  for (int g = threadIdx.x; g < r.npwx; g += NT) {
    cplx<T> h = zero;
    if (g < r.npw) {
      int gm = r.gmap[g];
      h = lds_ld(Z + (gm >> 8) * ZS + (gm & 255));
      cplx<T> v = r.p[g];
      T kk = (T)r.kin[g];
      h.x += kk * v.x;
      h.y += kk * v.y;
      for (int q = 0; q < nproj; ++q) h = cfma(r.bk[(long)q * r.npwx + g], lds_ld(gam + q), h);
    }
    r.hp[g] = h;
  }
}

// ---------------------------------------------------------------- 1D passes
// Each pass comes in a one-work-item-per-line form and, for even N, a
// lane-pair form (pair_inverse / pair_forward in fft.hpp).  The callbacks
// work on register slots: inverse outputs go to st(J, v) for slot J, which is
// point J of the line (one work-item) or point 2 J + h (lane h of a pair);
// forward inputs come from ld(J) for the same slots; forward outputs go to
// st(K, v), K < min(WC, N/2) for a pair, which is coefficient K or K + h N/2.
// The callers turn slots into addresses with per-lane bases and uniform
// strides.

// inverse along one line: WC inputs from ld(m) -> N outputs
template <class T, int N, int WC, bool PAIR, class LD, class ST>
__device__ __forceinline__ void line_inverse(int h, LD&& ld, ST&& st) {
  if constexpr (PAIR) {
    constexpr int M = N / 2;
    cplx<T> v[M];
    pair_inverse<T, N, WC, +1>(v, h, ld);
    sfor<M>([&](auto j) { st(decltype(j)::value, v[decltype(j)::value]); });
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

// forward along one line: N inputs -> the first WC outputs
template <class T, int N, int WC, bool PAIR, class LD, class ST>
__device__ __forceinline__ void line_forward(int h, LD&& ld, ST&& st) {
  if constexpr (PAIR) {
    constexpr int M = N / 2;
    constexpr int KO = WC < M ? WC : M;
    cplx<T> v[M];
    sfor<M>([&](auto j) { v[decltype(j)::value] = ld(decltype(j)::value); });
    pair_forward<T, N, WC, -1>(v, h);
    sfor<KO>([&](auto k) { st(decltype(k)::value, v[decltype(k)::value]); });
  } else {
    cplx<T> v[N];
    sfor<N>([&](auto j) { v[decltype(j)::value] = ld(decltype(j)::value); });
    fft<T, N, -1>(v);
    sfor<WC>([&](auto j) { st(decltype(j)::value, v[decltype(j)::value]); });
  }
}

// x line: WC inputs -> N points -> * V/N_r -> forward -> WC outputs; vat(J)
// gives V at the point of slot J
template <class T, int N, int WC, bool PAIR, class LD, class VAT, class ST>
__device__ __forceinline__ void line_xv(int h, LD&& ld, VAT&& vat, ST&& st) {
  if constexpr (PAIR) {
    constexpr int M = N / 2;
    constexpr int KO = WC < M ? WC : M;
    cplx<T> v[M];
    pair_inverse<T, N, WC, +1>(v, h, ld);
    sfor<M>([&](auto j) {
      constexpr int J = decltype(j)::value;
      T f = vat(J);
      v[J].x *= f;
      v[J].y *= f;
    });
    pair_forward<T, N, WC, -1>(v, h);
    sfor<KO>([&](auto k) { st(decltype(k)::value, v[decltype(k)::value]); });
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

// Global loads through a buffer descriptor: a per-lane byte offset plus a
// wave-uniform one, so that strided loads cost no vector address arithmetic.
// Offsets past num_records read as zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, 0x00020000);
}
template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}

// ---------------------------------------------------------------- the kernel
// LDS layout of one workgroup, in elements of cplx<T> unless noted.
struct HpsiLds {
  size_t z, y, red, gam, dl, sof_bytes, bytes;
};
template <class T, int N, int WC>
__host__ __device__ inline HpsiLds hpsi_lds_layout(int smax, int wx, int l3c, int nproj, int threads) {
  const size_t cs = sizeof(cplx<T>);
  const int np = nproj > 0 ? nproj : 1;
  HpsiLds L;
  L.z = (size_t)(smax + 2) * (N | 1);  // sticks, then one zero row and one write-sink row
  L.y = (size_t)l3c * wx * (N | 1);    // slab planes: [l3c][wx][N | 1]
  L.red = (size_t)(threads / 64) * np; // per-wave projector partial sums
  L.gam = np;
  L.dl = (size_t)np * np;
  L.sof_bytes = (size_t)2 * wx * WC * sizeof(int);  // stick row offsets for reads and for writes
  L.bytes = (L.z + L.y + L.red + L.gam + L.dl) * cs + L.sof_bytes;
  return L;
}

// ZYP: z and y passes in lane pairs; XP: x pass in lane pairs (even N only).
// XC: each x line as one convolution over the window instead (XP unused).
// WC: compile-time capacity of the Miller window along each axis (>= the
// actual extents wx, wy, wz); entries beyond the actual window are zero.
// NT: work-items per workgroup (256, 512 or 1024).
// vr: V/N_r permuted per slab width (Vp[slab][l1][lc][l2]); with XC the x
// taps of V/N_r instead (xtaps_kernel).
template <class T, int N, int WC, bool ZYP, bool XP, int NT, bool XC = false>
__global__ __launch_bounds__(NT) void hpsi_kernel(KTables t, VecSel sel, int nproj,
                                                  const cplx<T>* __restrict__ beta,
                                                  const cplx<T>* __restrict__ dij,
                                                  const T* __restrict__ vr,
                                                  const cplx<T>* __restrict__ psi,
                                                  cplx<T>* __restrict__ hpsi, int l3c, int per_xcd,
                                                  int ntask) {
  static_assert(!(ZYP || XP) || N % 2 == 0, "lane-pair passes need an even length");
  static_assert(!XC || WC < N, "the x convolution is for windows narrower than the mesh");
  Row<T> r;
  if (!row_of_block(t, sel, nproj, beta, psi, hpsi, per_xcd, ntask, r)) return;
  const int wx = t.wx, wy = t.wy;
  const int ns = r.ns;
  constexpr int ZS = N | 1;  // stick row stride (odd: no LDS bank aliasing between sticks)
  constexpr int NW = NT / 64;
  const int zrow = t.smax, sink = t.smax + 1;  // all-zero stick, write-only stick

  const HpsiLds L = hpsi_lds_layout<T, N, WC>(t.smax, wx, l3c, nproj, NT);
  extern __shared__ __align__(16) unsigned char smem[];
  typedef lds_t<cplx<T>> lc;
  lc* Z = (lc*)smem;     // [smax + 2][ZS]
  lc* Y = Z + L.z;       // [l3c][wx][YS]: the y lines of the slab's occupied x columns
  lc* red = Y + L.y;     // [NW][nproj]
  lc* gam = red + L.red;  // [nproj]
  lc* dl = gam + L.gam;   // [nproj][nproj]
  // byte offset in Z of the stick of (m1', m2'), [wx][WC]: the zero row where
  // there is none (for reads), the write-only row (for writes)
  lds_t<int>* sofr = (lds_t<int>*)(dl + L.dl);
  lds_t<int>* sofw = sofr + wx * WC;
  constexpr int YS = N | 1;  // y-line stride in Y (odd: no bank aliasing between columns)
  constexpr int CS = (int)sizeof(cplx<T>);

  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int h0 = tid & 1;
  const cplx<T> zero = {T(0), T(0)};
  constexpr int kZyStride = ZYP ? NT / 2 : NT;
  constexpr int kXStride = XP ? NT / 2 : NT;
  const int zy_slot = ZYP ? tid >> 1 : tid;
  const int x_slot = XP ? tid >> 1 : tid;

  // ---- 0. start the loads of the first plane waves of this work-item (psi,
  //         map, first projectors) so that they arrive during the zeroing
  constexpr int kPre = 2;
  const int npre = min(nproj, kProjChunk);
  cplx<T> pv[kPre], bv[kPre][kProjChunk];
  int gv[kPre];
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int g = tid + u * NT;
    if (g < r.npw) {
      pv[u] = r.p[g];
      gv[u] = r.gmap[g];
#pragma unroll
      for (int q = 0; q < kProjChunk; ++q)
        if (q < npre) bv[u][q] = r.bk[(long)q * r.npwx + g];
    }
  }

  // ---- 1. zero the stick windows and the zero row, stage the stick map and D
  for (int i = tid; i < ns * WC; i += NT) {
    int s = i / WC, j = i - s * WC;
    lds_st(Z + s * ZS + j, zero);
  }
  for (int i = tid; i < N; i += NT) lds_st(Z + zrow * ZS + i, zero);
  for (int i = tid; i < wx * WC; i += NT) {
    const int m1 = i / WC, m2 = i - m1 * WC;
    int s = m2 < wy ? r.sof[m1 * wy + m2] : -1;
    sofr[i] = (s >= 0 ? s : zrow) * ZS * CS;
    sofw[i] = (s >= 0 ? s : sink) * ZS * CS;
  }
  for (int i = tid; i < nproj * nproj; i += NT) lds_st(dl + i, dij[i]);
  __syncthreads();

  // ---- 2. scatter psi into the sticks; the same loads give the partial
  //         projector overlaps lambda_q = sum_G beta_q^* psi (Eq. lambdah),
  //         summed over each wave into red[wave][q]
  {
    T ax[kProjChunk], ay[kProjChunk];
    auto acc = [&](int q, cplx<T> b, cplx<T> v) {  // += conj(b) * v
      ax[q] = fma_t(b.y, v.y, fma_t(b.x, v.x, ax[q]));
      ay[q] = fma_t(-b.y, v.x, fma_t(b.x, v.y, ay[q]));
    };
    auto flush = [&](int q0) {
#pragma unroll
      for (int q = 0; q < kProjChunk; ++q) {
        if (q0 + q < nproj) {
          const T sx = wave_sum(ax[q]), sy = wave_sum(ay[q]);
          if (lane == 0) lds_st(red + wave * nproj + q0 + q, cplx<T>{sx, sy});
        }
      }
    };
#pragma unroll
    for (int q = 0; q < kProjChunk; ++q) ax[q] = ay[q] = T(0);
#pragma unroll
    for (int u = 0; u < kPre; ++u) {
      if (tid + u * NT < r.npw) {
        lds_st(Z + (gv[u] >> 8) * ZS + (gv[u] & 255), pv[u]);
#pragma unroll
        for (int q = 0; q < kProjChunk; ++q)
          if (q < npre) acc(q, bv[u][q], pv[u]);
      }
    }
    for (int g = tid + kPre * NT; g < r.npw; g += NT) {
      const cplx<T> v = r.p[g];
      const int gm = r.gmap[g];
      lds_st(Z + (gm >> 8) * ZS + (gm & 255), v);
#pragma unroll
      for (int q = 0; q < kProjChunk; ++q)
        if (q < npre) acc(q, r.bk[(long)q * r.npwx + g], v);
    }
    flush(0);
    for (int q0 = kProjChunk; q0 < nproj; q0 += kProjChunk) {  // more than kProjChunk projectors
#pragma unroll
      for (int q = 0; q < kProjChunk; ++q) ax[q] = ay[q] = T(0);
      for (int g = tid; g < r.npw; g += NT) {
        const cplx<T> v = r.p[g];
#pragma unroll
        for (int q = 0; q < kProjChunk; ++q)
          if (q0 + q < nproj) acc(q, r.bk[(long)(q0 + q) * r.npwx + g], v);
      }
      flush(q0);
    }
  }
  __syncthreads();

  // ---- 3. inverse z on the sticks (W -> N), on as few waves as hold them;
  //         gamma = D lambda on the last wave
  {
    const int zlanes = (ZYP ? 2 : 1) * ns;
    const int zwaves = min(NW, (zlanes + 63) / 64);
    if (wave < zwaves) {
      for (int s = zy_slot; s < ns; s += (ZYP ? zwaves * 32 : zwaves * 64)) {
        const int h = lane_half(h0);
        lc* zr = Z + s * ZS;
        lc* zh = zr + (ZYP ? h : 0);
        line_inverse<T, N, WC, ZYP>(
            h, [&](int m) { return lds_ld(zr + m); }, [&](int j, cplx<T> v) { lds_st(zh + (ZYP ? 2 : 1) * j, v); });
      }
    }
    // read by the gather; the barriers of the slab loop publish it
    if (wave == NW - 1 && lane < nproj) finish_gamma(lane, nproj, dl, red, NW, gam);
  }
  __syncthreads();

  // ---- 4. slabs of z planes.  V is stored permuted per slab so that the
  //         x-line work-items of a slab read it contiguously: Vp[slab][l1][lc][l2].
  const __amdgpu_buffer_rsrc_t vres = make_rsrc(vr, N * N * N * (int)sizeof(T));
  for (int l30 = 0; l30 < N; l30 += l3c) {
    const int nl = min(l3c, N - l30);
    const int vbase = l30 * N * N * (int)sizeof(T);  // byte offset of the slab in V
    // inverse y on the occupied columns m1' < wx: W inputs (from the sticks) -> N outputs
    for (int i = zy_slot; i < wx * nl; i += kZyStride) {
      const int h = lane_half(h0);
      const int lcn = i / wx, m1 = i - lcn * wx, l3 = l30 + lcn;
      lc* yh = Y + i * YS + (ZYP ? h : 0);  // i = lc wx + m1
      const lds_t<int>* so = sofr + m1 * WC;
      const lds_t<char>* zl = (const lds_t<char>*)(Z + l3);
      line_inverse<T, N, WC, ZYP>(
          h, [&](int m) { return lds_ld((const lc*)(zl + so[m])); },
          [&](int j, cplx<T> v) { lds_st(yh + (ZYP ? 2 : 1) * j, v); });
    }
    __syncthreads();
    if constexpr (XC) {
      // x lines as convolutions: the inverse transform along x, the product
      // with V/N_r and the forward transform along x of one line together are
      // out(m') = sum_m X[m' - m] in(m) over the window (Eqs. xfft, fwFFT),
      // X[d] = sum_l1 V(l1)/N_r exp(-2 pi i d l1 / N) the line's taps, read
      // from xt[l3][d + WC - 1][l2]; a work-item owns one line, in place
      constexpr int DW = 2 * WC - 1;
      // the compact x convolution holds about 100 fewer registers; it is the
      // faster one in FP32 and in the FP64 kernels of 512 work-items (36^3,
      // capacity 11: 4.09 against 4.16 ms on 1728 k), and it keeps the
      // 1024-work-item kernels from spilling, while the FP64 ones at 256
      // work-items run faster with every tap loaded up front (30^3: 1.91
      // against 1.94 ms on 2048 k)
      constexpr bool XCOMPACT = sizeof(T) == 4 || NT >= 512;
      const cplx<T>* xt = reinterpret_cast<const cplx<T>*>(vr);
      for (int i = tid; i < N * nl; i += NT) {
        const int lcn = i / N, l2 = i - lcn * N;
        lc* y = Y + lcn * wx * YS + l2;
        const cplx<T>* tp = xt + (long)(l30 + lcn) * DW * N + l2;
        if constexpr (XCOMPACT) {
        // compact form: the inputs m in order, each read from LDS and added
        // into the outputs with the taps X[m' - m], so that only the outputs,
        // the input and the WC taps in use are live: a tap enters at the
        // first input that reaches it (every tap for m = 0, then the tap of
        // the first output) and leaves WC inputs later; a scheduling fence
        // per input keeps the compiler from loading ahead.  The line is
        // transformed in place, so all its outputs are formed before any is
        // stored.  (The arrays live in a lambda of their own: declared in the
        // loop body they come out with 55 more registers and spills.)
        [&] {
        cplx<T> out[WC], tap[DW];
        sfor<WC>([&](auto o) { out[decltype(o)::value] = zero; });
        sfor<WC>([&](auto mm) {
          constexpr int M = decltype(mm)::value;
          if (M < wx) {
            const cplx<T> x = lds_ld(y + M * YS);
            sfor<WC>([&](auto o) {
              constexpr int MP = decltype(o)::value;
              constexpr int DD = MP - M + (WC - 1);  // tap index of m' - m
              if constexpr (M == 0 || MP == 0) tap[DD] = tp[(long)DD * N];
              out[MP] = cfma(tap[DD], x, out[MP]);
            });
          }
          __builtin_amdgcn_sched_barrier(0);
        });
        sfor<WC>([&](auto o) {
          constexpr int MP = decltype(o)::value;
          if (MP < wx) lds_st(y + MP * YS, out[MP]);
        });
        }();
        } else {
        // all taps at once: the inputs and outputs in registers, every tap
        // loaded once and applied to the outputs it reaches
        cplx<T> in[WC], out[WC];
        sfor<WC>([&](auto mm) {
          constexpr int M = decltype(mm)::value;
          in[M] = M < wx ? lds_ld(y + M * YS) : zero;
          out[M] = zero;
        });
        sfor<DW>([&](auto dd) {
          constexpr int DD = decltype(dd)::value;
          constexpr int D = DD - (WC - 1);  // m' - m
          const cplx<T> tap = tp[(long)DD * N];
          sfor<WC>([&](auto mp) {
            constexpr int MP = decltype(mp)::value;
            constexpr int M = MP - D;
            if constexpr (M >= 0 && M < WC) out[MP] = cfma(tap, in[M], out[MP]);
          });
        });
        sfor<WC>([&](auto mm) {
          constexpr int M = decltype(mm)::value;
          if (M < wx) lds_st(y + M * YS, out[M]);
        });
        }
      }
    } else {
    // x lines: W inputs -> N points -> * V/N_r -> forward -> W outputs
    for (int i = x_slot; i < N * nl; i += kXStride) {
      const int h = lane_half(h0);
      const int lcn = i / N, l2 = i - lcn * N;  // i = lc N + l2
      lc* y = Y + lcn * wx * YS + l2;
      const int mo = XP ? h * (N / 2) : 0;
      lc* yo = y + mo * YS;
      // V at point l1 of this line: byte vbase + ((l1 nl + lc) N + l2) sizeof(T)
      const int voff = (i + (XP ? h : 0) * nl * N) * (int)sizeof(T);
      const int vstep = (XP ? 2 : 1) * nl * N * (int)sizeof(T);
      line_xv<T, N, WC, XP>(
          h, [&](int m) { return m < wx ? lds_ld(y + m * YS) : zero; },
          [&](int j) { return buf_load<T>(vres, voff, vbase + j * vstep); },
          [&](int k, cplx<T> v) {
            if (k + mo < wx) lds_st(yo + k * YS, v);
          });
    }
    }
    __syncthreads();
    // forward y: N inputs -> W outputs, back into the sticks (outputs with no
    // stick go to the write-only row)
    for (int i = zy_slot; i < wx * nl; i += kZyStride) {
      const int h = lane_half(h0);
      const int lcn = i / wx, m1 = i - lcn * wx, l3 = l30 + lcn;
      const lc* yh = Y + i * YS + (ZYP ? h : 0);
      const int mo = ZYP ? h * (N / 2) : 0;
      const lds_t<int>* so = sofw + m1 * WC + mo;
      lds_t<char>* zl = (lds_t<char>*)(Z + l3);
      line_forward<T, N, WC, ZYP>(
          h, [&](int j) { return lds_ld(yh + (ZYP ? 2 : 1) * j); },
          [&](int k, cplx<T> v) {
            // the second lane of a pair also returns outputs N/2.. of the line
            if (k + mo < WC) lds_st((lc*)(zl + so[k]), v);
          });
    }
    __syncthreads();
  }

  // ---- 5. forward z on the sticks: N inputs -> W outputs (in place)
  for (int s = zy_slot; s < ns; s += kZyStride) {
    const int h = lane_half(h0);
    lc* zr = Z + s * ZS;
    const int mo = ZYP ? h * (N / 2) : 0;
    line_forward<T, N, WC, ZYP>(
        h, [&](int j) { return lds_ld(zr + (ZYP ? 2 * j + h : j)); },
        [&](int k, cplx<T> v) {
          if (k + mo < WC) lds_st(zr + mo + k, v);
        });
  }
  __syncthreads();

  // ---- 6. gather + kinetic + nonlocal
  gather_add<T, ZS, NT>(r, nproj, Z, gam);
}

// ---------------------------------------------------------------- launching

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

// Taps of the x-line convolutions: xt[l3][d + wc - 1][l2] =
// sum_l1 v[l1][l2][l3] exp(-2 pi i d l1 / n) for |d| < wc, from V/N_r in FP64
// (then rounded to T).
template <class T>
__global__ void xtaps_kernel(const double* __restrict__ v, cplx<T>* __restrict__ xt, int n, int wc) {
  const int dw = 2 * wc - 1;
  const long total = (long)n * dw * n;
  for (long o = blockIdx.x * (long)blockDim.x + threadIdx.x; o < total; o += (long)gridDim.x * blockDim.x) {
    const int l2 = (int)(o % n);
    const long r = o / n;
    const int dd = (int)(r % dw), l3 = (int)(r / dw);
    const int d = ((dd - (wc - 1)) % n + n) % n;
    double sr = 0.0, si = 0.0;
    int ph = 0;  // d l1 mod n
    for (int l1 = 0; l1 < n; ++l1) {
      double sn, cs;
      sincospi(2.0 * ph / n, &sn, &cs);
      const double vv = v[((long)l1 * n + l2) * n + l3];
      sr += vv * cs;
      si -= vv * sn;
      ph += d;
      if (ph >= n) ph -= n;
    }
    xt[o] = {(T)sr, (T)si};
  }
}

// Shape of one launch: kernel variant (1 = one work-item per line, 2 = lane
// pair per line, even N only, 3 = lane pairs for the x lines only, 4 = one
// work-item per line with each x line as a convolution, 5 = lane pairs for
// the y and z lines with x convolutions; 4 and 5 for windows narrower than the
// mesh), slab width in z planes, work-items per workgroup.
struct HpsiShape {
  int variant = 1;
  int l3c = 1;
  int threads = 256;
};

// Autotuning results shared by every context of the process (hpsi.hip).
extern std::mutex g_hpsi_tune_mu;
extern std::map<std::vector<long>, HpsiShape> g_hpsi_tuned;

constexpr size_t kLdsPerCu = 160 * 1024;
constexpr long kTuneMinRows = 4096;  // smallest launch (in (k, band) rows) that is autotuned

template <class T, int N, int WC>
size_t hpsi_lds(const KTables& t, int l3c, int nproj, int threads) {
  return hpsi_lds_layout<T, N, WC>(t.smax, t.wx, l3c, nproj, threads).bytes;
}

// Workgroup sizes instantiated: 512 work-items leave 256 registers per lane
// and 1024 leave 128, so each is built only where the kernel fits without
// spilling (the double precision one-line-per-work-item passes need the full
// 512 from N = 30 on).
template <class T, int N, int VARIANT>
constexpr bool allow_512() {
  return !(sizeof(T) == 8 && VARIANT == 1 && N >= 30);
}
template <class T, int N, int VARIANT>
constexpr bool allow_1024() {
  if constexpr (VARIANT == 4) return sizeof(T) == 4 && N <= 24;
  if constexpr (VARIANT == 5) return true;
  return sizeof(T) == 4 ? (VARIANT != 1 || N <= 20) : VARIANT == 2;
}

template <class T, int N, int WC, int VARIANT>
const void* kernel_for(int threads) {
  // variant 1: one work-item per line; 2: lane pairs for every line;
  // 3: lane pairs for the x lines only (their registers set the occupancy);
  // 4: one work-item per line, x lines as convolutions; 5: lane pairs for the
  // y and z lines, x lines as convolutions
  constexpr bool ZYP = VARIANT == 2 || VARIANT == 5, XP = VARIANT == 2 || VARIANT == 3;
  constexpr bool XC = VARIANT >= 4;
  if constexpr (XC && WC >= N) {
    return nullptr;
  } else {
    if (threads == 256) return (const void*)hpsi_kernel<T, N, WC, ZYP, XP, 256, XC>;
    if constexpr (allow_512<T, N, VARIANT>()) {
      if (threads == 512) return (const void*)hpsi_kernel<T, N, WC, ZYP, XP, 512, XC>;
    }
    if constexpr (allow_1024<T, N, VARIANT>()) {
      if (threads == 1024) return (const void*)hpsi_kernel<T, N, WC, ZYP, XP, 1024, XC>;
    }
    return nullptr;
  }
}

template <class T, int N, int WC>
const void* hpsi_kernel_ptr(const HpsiShape& sh) {
  if constexpr (N % 2 == 0) {
    if (sh.variant == 2) return kernel_for<T, N, WC, 2>(sh.threads);
    if (sh.variant == 3) return kernel_for<T, N, WC, 3>(sh.threads);
    if (sh.variant == 5) return kernel_for<T, N, WC, 5>(sh.threads);
  }
  if (sh.variant == 1) return kernel_for<T, N, WC, 1>(sh.threads);
  if (sh.variant == 4) return kernel_for<T, N, WC, 4>(sh.threads);
  return nullptr;
}

// vscratch: caller-provided device memory of at least N^3 sizeof(T) bytes for
// the permuted potential, rebuilt on every launch (nothing is allocated);
// null: the context's own copy, built once per slab width.
template <class T, int N, int WC>
pw_status launch_shape(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st, HpsiShape sh,
                       void* vscratch = nullptr) {
  KTables t = c->tables();
  const int l3c = sh.l3c;
  const int nproj_k = c->have_proj ? c->nproj : 0;
  const size_t lds = hpsi_lds<T, N, WC>(t, l3c, nproj_k, sh.threads);
  const void* kern = hpsi_kernel_ptr<T, N, WC>(sh);
  if (!kern) return set_err(c, PW_EINVAL, "no H|psi> kernel for this variant and workgroup size");
  {
    pw_status s = ensure_lds_limit(c, kern, lds);
    if (s != PW_OK) return s;
  }
  const long ntask = (long)t.nk * sel.nvec;
  if (ntask <= 0) return PW_OK;
  if (ntask > (1L << 30)) return set_err(c, PW_EINVAL, "too many (k, band) rows in one call");
  const bool fp64 = sizeof(T) == 8;
  const T* v = (const T*)(fp64 ? (const void*)c->d_v64 : (const void*)c->d_v32);
  void* vp = vscratch;
  const size_t taps_bytes = (size_t)N * N * (2 * WC - 1) * sizeof(cplx<T>);
  if (sh.variant >= 4) {
    // x-line taps for this window capacity (rebuilt when it changes)
    if (vscratch) {
      hipLaunchKernelGGL(xtaps_kernel<T>, dim3(256), dim3(256), 0, st, c->d_v64, (cplx<T>*)vscratch, N, WC);
    } else {
      int& have = fp64 ? c->xtaps_wc64 : c->xtaps_wc32;
      void*& own = fp64 ? c->d_xtaps64 : c->d_xtaps32;
      if (have != WC || !own) {
        if (own && have != WC) {
          dev_free(c, own);
          own = nullptr;
        }
        if (!own) {
          pw_status s = dev_alloc(c, taps_bytes, &own);
          if (s != PW_OK) return s;
        }
        hipLaunchKernelGGL(xtaps_kernel<T>, dim3(256), dim3(256), 0, st, c->d_v64, (cplx<T>*)own, N, WC);
        have = WC;
      }
      vp = own;
    }
  } else if (vscratch) {
    hipLaunchKernelGGL(permute_v_kernel<T>, dim3(64), dim3(256), 0, st, v, (T*)vscratch, N, l3c);
  } else {
    // permuted potential for this slab width (rebuilt when the width changes)
    int& have = fp64 ? c->vperm_l3c64 : c->vperm_l3c32;
    void*& own = fp64 ? c->d_vperm64 : c->d_vperm32;
    if (have != l3c || !own) {
      if (!own) {
        pw_status s = dev_alloc(c, (size_t)N * N * N * sizeof(T), &own);
        if (s != PW_OK) return s;
      }
      hipLaunchKernelGGL(permute_v_kernel<T>, dim3(64), dim3(256), 0, st, v, (T*)own, N, l3c);
      have = l3c;
    }
    vp = own;
  }
  int per_xcd = (int)((ntask + 7) / 8);
  int nproj = c->have_proj ? c->nproj : 0;
  const cplx<T>* beta = (const cplx<T>*)(fp64 ? c->d_beta64 : c->d_beta32);
  const cplx<T>* dij = (const cplx<T>*)(fp64 ? c->d_dij64 : c->d_dij32);
  const T* vpt = (const T*)vp;
  const cplx<T>* pin = (const cplx<T>*)psi;
  cplx<T>* pout = (cplx<T>*)hpsi;
  int l3c_arg = l3c, ntask_arg = (int)ntask;
  VecSel sel_arg = sel;
  void* args[] = {&t, &sel_arg, &nproj, &beta, &dij, &vpt, &pin, &pout, &l3c_arg, &per_xcd, &ntask_arg};
  hipError_t e = hipLaunchKernel(kern, dim3(8u * (unsigned)per_xcd), dim3(sh.threads), args, lds, st);
  if (e == hipSuccess) e = hipGetLastError();
  if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string("h_psi launch: ") + hipGetErrorString(e));
  c->last_hpsi_variant = sh.variant;
  c->last_hpsi_slab = sh.l3c;
  c->last_hpsi_threads = sh.threads;
  if (c->trace) {
    e = hipStreamSynchronize(st);
    if (e != hipSuccess) return set_err(c, PW_EDEVICE, std::string("h_psi: ") + hipGetErrorString(e));
  }
  return PW_OK;
}

// Workgroups of this kernel one CU can hold by registers (4 SIMDs with 512
// VGPRs per lane, allocated in blocks of 8); 0 if the kernel spills registers
// to scratch memory (left out of the autotuning).
inline int wgs_by_vgpr(const void* kern, int threads) {
  int regs = 0;
  size_t scratch = 0;
  if (!kernel_resources(kern, &regs, &scratch) || regs <= 0) return 1;
  if (scratch > 0) return 0;
  const int v = (regs + 7) / 8 * 8;
  const int waves_per_simd = std::min(8, 512 / v);
  return std::max(1, waves_per_simd * 4 / (threads / 64));
}

// Candidate shapes: for each variant and workgroup size, the whole mesh as one
// slab, and the widest slab that fits in the LDS share for 1, 2 or 3
// workgroups per CU (as many as the registers allow), capped where every x
// line already has its own work-item (or lane pair); and, for one workgroup
// per CU, every slab width that splits the mesh evenly into a different
// number of slabs (ceil(N / s) planes) and fits: the number of slabs sets how
// many y passes run and how the x lines fill the work-items in the last round
// of each slab, which no single width balances for every mesh.
template <class T, int N, int WC>
std::vector<HpsiShape> hpsi_candidates(const KTables& t, int nproj) {
  std::vector<HpsiShape> out;
  for (int variant : {1, 2, 3, 4, 5}) {
    if ((variant == 2 || variant == 3 || variant == 5) && N % 2) continue;
    for (int threads : {256, 512, 1024}) {
      const void* kern = hpsi_kernel_ptr<T, N, WC>({variant, 1, threads});
      if (!kern) continue;
      const int lanes = (variant == 2 || variant == 3) ? 2 : 1;  // work-items per x line
      const int cap = std::min(N, std::max(1, threads / (lanes * N)));
      const int max_wg = std::min(3, wgs_by_vgpr(kern, threads));  // 0: spills, skipped
      // the whole mesh in one slab, and for 1..max_wg workgroups per CU the
      // widest slab up to one x line per work-item that fits their LDS share
      for (int wg = 0; wg <= max_wg; ++wg) {
        if (max_wg == 0) break;
        const size_t share = kLdsPerCu / (wg ? wg : 1);
        int l3c = wg == 0 ? N : cap;
        while (l3c > 1 && hpsi_lds<T, N, WC>(t, l3c, nproj, threads) > share) --l3c;
        if (hpsi_lds<T, N, WC>(t, l3c, nproj, threads) > kLdsPerCu) continue;
        bool dup = false;
        for (auto& o : out) dup = dup || (o.variant == variant && o.l3c == l3c && o.threads == threads);
        if (!dup) out.push_back({variant, l3c, threads});
      }
      if (max_wg == 0) continue;
      for (int nslab = 2; nslab <= 6; ++nslab) {
        const int l3c = (N + nslab - 1) / nslab;
        if (l3c * lanes * N < threads / 2) break;  // x lines would leave most work-items idle
        if (hpsi_lds<T, N, WC>(t, l3c, nproj, threads) > kLdsPerCu) continue;
        bool dup = false;
        for (auto& o : out) dup = dup || (o.variant == variant && o.l3c == l3c && o.threads == threads);
        if (!dup) out.push_back({variant, l3c, threads});
      }
    }
  }
  return out;
}

template <class T, int N, int WC>
pw_status launch_one(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st, void* vscratch) {
  KTables t = c->tables();
  const int nproj = c->have_proj ? c->nproj : 0;
  if (c->hpsi_variant != 0 || c->hpsi_slab != 0 || c->hpsi_threads != 0) {  // explicit shape
    if ((c->hpsi_variant == 2 || c->hpsi_variant == 3 || c->hpsi_variant == 5) && N % 2)
      return set_err(c, PW_EINVAL, "lane-pair variants need an even mesh");
    HpsiShape sh;
    sh.variant = c->hpsi_variant ? (int)c->hpsi_variant : 1;
    sh.threads = c->hpsi_threads ? (int)c->hpsi_threads : 256;
    if (!hpsi_kernel_ptr<T, N, WC>(sh))
      return set_err(c, PW_EINVAL, "no H|psi> kernel for this variant and workgroup size on this mesh");
    const int lanes = (sh.variant == 2 || sh.variant == 3) ? 2 : 1;
    sh.l3c = c->hpsi_slab ? (int)std::min<int64_t>(c->hpsi_slab, N)
                          : std::min(N, std::max(1, sh.threads / (lanes * N)));
    if (!c->hpsi_slab)
      while (sh.l3c > 1 && hpsi_lds<T, N, WC>(t, sh.l3c, nproj, sh.threads) > kLdsPerCu) --sh.l3c;
    if (hpsi_lds<T, N, WC>(t, sh.l3c, nproj, sh.threads) > kLdsPerCu)
      return set_err(c, PW_EINVAL, "requested H|psi> slab does not fit in LDS");
    return launch_shape<T, N, WC>(c, sel, psi, hpsi, st, sh, vscratch);
  }
  // autotune once per (precision, mesh, window capacity, row-count bucket);
  // launches of fewer rows than kTuneMinRows are not worth timing and take the
  // shape tuned for the smallest bucket seen, else a fixed default
  long rows = kTuneMinRows;
  while (rows < (long)t.nk * sel.nvec) rows <<= 1;
  const std::vector<long> key = {(long)sizeof(T), N, WC, rows};
  auto fits = [&](HpsiShape& sh) {  // narrow the slab to this context's LDS need
    while (sh.l3c > 1 && hpsi_lds<T, N, WC>(t, sh.l3c, nproj, sh.threads) > kLdsPerCu) --sh.l3c;
    return hpsi_lds<T, N, WC>(t, sh.l3c, nproj, sh.threads) <= kLdsPerCu;
  };
  {
    std::lock_guard<std::mutex> lk(g_hpsi_tune_mu);
    auto it = g_hpsi_tuned.find(key);
    if (it == g_hpsi_tuned.end() && (long)t.nk * sel.nvec < kTuneMinRows) {
      for (auto jt = g_hpsi_tuned.begin(); jt != g_hpsi_tuned.end(); ++jt)
        if (jt->first[0] == (long)sizeof(T) && jt->first[1] == N && jt->first[2] == WC) {
          it = jt;  // the map orders keys, so this is the smallest bucket
          break;
        }
    }
    if (it != g_hpsi_tuned.end()) {
      HpsiShape sh = it->second;
      if (fits(sh)) return launch_shape<T, N, WC>(c, sel, psi, hpsi, st, sh, vscratch);
    }
  }
  // small launches, and launches that may not allocate (the tuning times
  // candidates with events and builds their potentials), take a fixed shape
  if ((long)t.nk * sel.nvec < kTuneMinRows || vscratch) {
    HpsiShape sh;
    sh.variant = (N % 2 == 0 && N >= 30) ? 2 : 1;
    sh.threads = sh.variant == 2 ? 512 : 256;
    sh.l3c = std::min(N, std::max(1, sh.threads / ((sh.variant == 2 ? 2 : 1) * N)));
    while (sh.l3c > 1 && hpsi_lds<T, N, WC>(t, sh.l3c, nproj, sh.threads) > kLdsPerCu / 2) --sh.l3c;
    if (!fits(sh)) return set_err(c, PW_EINVAL, "H|psi> working set does not fit in LDS for this mesh");
    return launch_shape<T, N, WC>(c, sel, psi, hpsi, st, sh, vscratch);
  }
  auto cands = hpsi_candidates<T, N, WC>(t, nproj);
  if (cands.empty()) return set_err(c, PW_EINVAL, "H|psi> working set does not fit in LDS for this mesh");
  HpsiShape sh = cands[0];
  if (cands.size() > 1) {
    // two rounds: every candidate once (one warm-up launch, which also builds
    // what it reads of the potential, then one timed), then the three fastest
    // again with four timed launches each
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
      (void)hipGetLastError();
      return set_err(c, PW_EDEVICE, "hipEventCreate failed");
    }
    pw_status s = PW_OK;
    auto time_it = [&](const HpsiShape& cand, int reps, float* ms) {
      if ((s = launch_shape<T, N, WC>(c, sel, psi, hpsi, st, cand)) != PW_OK) return false;
      (void)hipEventRecord(e0, st);
      for (int r = 0; r < reps; ++r)
        if ((s = launch_shape<T, N, WC>(c, sel, psi, hpsi, st, cand)) != PW_OK) return false;
      (void)hipEventRecord(e1, st);
      (void)hipEventSynchronize(e1);
      (void)hipEventElapsedTime(ms, e0, e1);
      *ms /= reps;
      return true;
    };
    std::vector<std::pair<float, size_t>> t1;
    for (size_t i = 0; i < cands.size(); ++i) {
      float ms = 0.f;
      if (!time_it(cands[i], 1, &ms)) break;
      t1.push_back({ms, i});
      if (c->tune_log)
        fprintf(stderr, "hpsi tune fp%d N=%d WC=%d variant=%d threads=%d slab=%d: %.4f ms\n", (int)sizeof(T) * 8,
                N, WC, cands[i].variant, cands[i].threads, cands[i].l3c, ms);
    }
    if (s == PW_OK) {
      std::sort(t1.begin(), t1.end());
      float best = 1e30f;
      for (size_t j = 0; j < std::min<size_t>(3, t1.size()); ++j) {
        float ms = 0.f;
        if (!time_it(cands[t1[j].second], 4, &ms)) break;
        if (ms < best) {
          best = ms;
          sh = cands[t1[j].second];
        }
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != PW_OK) return s;
  }
  {
    std::lock_guard<std::mutex> lk(g_hpsi_tune_mu);
    g_hpsi_tuned[key] = sh;
  }
  return launch_shape<T, N, WC>(c, sel, psi, hpsi, st, sh);
}

// Window capacities built for an N^3 mesh: one below the first rung, then
// every other value from about N/3 to N/2 + 2 (the usual range of the
// wave-function window on a density-sized mesh), then N.  A launch takes the
// smallest one that holds the window, so at most one padded input per line is
// transformed, and none at the lowest rungs, where the window of a
// density-sized mesh most often falls (a padded input of the x convolution
// costs 2 WC - 1 of its WC^2 multiply-adds).
template <int N>
constexpr int wc_first() {
  return (N + 2) / 3 > 5 ? (N + 2) / 3 : 5;
}
template <int N, int WC>
constexpr int wc_next() {
  return WC >= N / 2 + 2 ? N : (WC + 2 < N / 2 + 2 ? WC + 2 : N / 2 + 2);
}

template <class T, int N, int WC>
pw_status launch_ladder(pw_ctx* c, int w, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st,
                        void* vscratch) {
  if constexpr (WC >= N) {
    return launch_one<T, N, N>(c, sel, psi, hpsi, st, vscratch);
  } else {
    if (w <= WC) return launch_one<T, N, WC>(c, sel, psi, hpsi, st, vscratch);
    return launch_ladder<T, N, wc_next<N, WC>()>(c, w, sel, psi, hpsi, st, vscratch);
  }
}

// H|psi> on an N^3 mesh
template <class T, int N>
pw_status launch_n(pw_ctx* c, const VecSel& sel, const void* psi, void* hpsi, hipStream_t st, void* vscratch) {
  const int w = std::max(c->wx, std::max(c->wy, c->wz));
  constexpr int W0 = wc_first<N>() - 1;
  if constexpr (W0 >= 5) {
    if (w <= W0) return launch_one<T, N, W0>(c, sel, psi, hpsi, st, vscratch);
  }
  return launch_ladder<T, N, wc_first<N>()>(c, w, sel, psi, hpsi, st, vscratch);
}

// one translation unit per mesh size instantiates both precisions; the
// dispatcher only declares them
#define MKPW_HPSI_INSTANTIATE(N)                                                                            \
  template pw_status launch_n<double, N>(pw_ctx*, const VecSel&, const void*, void*, hipStream_t, void*); \
  template pw_status launch_n<float, N>(pw_ctx*, const VecSel&, const void*, void*, hipStream_t, void*);
#define MKPW_HPSI_EXTERN(N)                                                                                        \
  extern template pw_status launch_n<double, N>(pw_ctx*, const VecSel&, const void*, void*, hipStream_t, void*); \
  extern template pw_status launch_n<float, N>(pw_ctx*, const VecSel&, const void*, void*, hipStream_t, void*);

}  // namespace mkpw
