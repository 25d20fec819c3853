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
//     k's bands, on the FP64 matrix cores;
//   * drho accumulates, per k, M(G1, G2) = sum_nu conj(u(G1)) du(G2) (16 x 16
//     tiles on the FP64 matrix cores) into bins of the Miller difference
//     d = m_G2 - m_G1 held in LDS; the per-k bins are summed over k
//     into the mesh (d mod N; 64 chunks of k summed in parallel, then the
//     chunks in a fixed order; the per-k bins themselves are summed with LDS
//     atomics, so results agree to rounding between runs, not bit for bit)
//     and one inverse transform of the mesh gives
//     drho(r) = sum_d F(d) exp(2 pi i d.l / N).
// The transforms of the single mesh (dV(r) -> dV~ with 1/N_r, F -> drho(r))
// are separable direct sums, one launch per axis.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
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


// The FP64 matrix cores: D (16 x 16) += A (16 x 4) B (4 x 16), one wave.  A
// lane l holds A[l % 16][l / 16] and B[l / 16][l % 16]; the result element
// D[4 r + l / 16][l % 16] is component r of the lane's accumulator.
typedef double mf64x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ mf64x4 mfma_16x16x4(double a, double b, mf64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Linear offset of a Miller triple in a box of sizes (., s2, s3): m1 s2 s3 +
// m2 s3 + m3.  Differences of such offsets are offsets of Miller differences,
// so a pair's position in a box that holds every difference is one subtraction.
__device__ __forceinline__ int miller_lin(int key, int s2, int s3) {
  int a, b, c;
  unpack_miller(key, a, b, c);
  return (a * s2 + b) * s3 + c;
}

// The transformed perturbation laid out over the box of Miller differences
// [lo, lo + sz) on each axis: box(d) = dvt(d mod N), so that no index of the
// pair sum needs a wrap
__global__ __launch_bounds__(256) void dv_box_kernel(const cd* __restrict__ dvt, int n1, int n2, int n3, int lo1,
                                                     int lo2, int lo3, int s1, int s2, int s3, cd* __restrict__ box) {
  const long e = (long)blockIdx.x * 256 + threadIdx.x;
  if (e >= (long)s1 * s2 * s3) return;
  const int i3 = (int)(e % s3), i2 = (int)((e / s3) % s2), i1 = (int)(e / ((long)s2 * s3));
  box[e] = dvt[((long)wrap(lo1 + i1, n1) * n2 + wrap(lo2 + i2, n2)) * n3 + wrap(lo3 + i3, n3)];
}

// rows of psi (nk, nbnd, npwx) with each k's plane waves put in the order
// perm[k] lists (zero past npw[k])
__global__ __launch_bounds__(256) void permute_rows_kernel(const cd* __restrict__ psi, const int* __restrict__ perm,
                                                           const int* __restrict__ npw, int npwx, int nbnd,
                                                           cd* __restrict__ out) {
  const int k = blockIdx.y;
  const long row = (long)k * nbnd;
  const int n = npw[k];
  const int* pk = perm + (long)k * npwx;
  for (long e = (long)blockIdx.x * 256 + threadIdx.x; e < (long)nbnd * npwx; e += (long)gridDim.x * 256) {
    const int b = (int)(e / npwx), g = (int)(e - (long)b * npwx);
    out[(row + b) * npwx + g] = g < n ? psi[(row + b) * npwx + pk[g]] : cd{0.0, 0.0};
  }
}

constexpr int kDvWaves = 4;  // waves per workgroup of dvpsi_mfma_kernel

// One chunk of U steps of four plane waves for dvpsi_mfma_kernel: this lane's
// L entry for each step (gathered from the box) and its B values (from the
// block of psi staged in LDS: row j of `bl` holds plane waves [b0, b0 + KC)
// of the lane's band of group j, real and imaginary parts interleaved, `part`
// already added, so plane wave g is element 2 (g - b0)), all loads of the
// chunk issued before its products (U is chosen so that a chunk holds 16
// products).  In the last, partial chunk (TAIL) a plane wave past the k
// sphere reads element 0 and box offset 0 and its L entry is zeroed, which
// removes its term; a band or row out of range only feeds results that are
// never stored.
template <int NG, int U, bool TAIL>
__device__ __forceinline__ void dv_chunk_lds(const cd* __restrict__ box, const int* wcol, int prow, int nin, int g0,
                                             int b0, int kq, const double* const (&bl)[NG], mf64x4 (&d1)[NG],
                                             mf64x4 (&d2)[NG]) {
  int w[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int g = g0 + 4 * u + kq;
    w[u] = wcol[TAIL && g >= nin ? 0 : g];
  }
  cd a[U];
  double bv[U][NG];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int g = g0 + 4 * u + kq;
    const int gl = TAIL && g >= nin ? 0 : g - b0;
    a[u] = box[prow + w[u]];
#pragma unroll
    for (int j = 0; j < NG; ++j) bv[u][j] = bl[j][2 * gl];
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    double xr = a[u].x, xi = a[u].y;
    if (TAIL && g0 + 4 * u + kq >= nin) xr = xi = 0.0;
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      d1[j] = mfma_16x16x4(xr, bv[u][j], d1[j]);
      d2[j] = mfma_16x16x4(xi, bv[u][j], d2[j]);
    }
  }
}

// plane waves of psi staged in LDS per step of dvpsi_mfma_kernel: 8 NG bands
// x kDvKC(NG) plane waves, 33 KiB for two buffers whatever NG
__host__ __device__ constexpr int dv_kc(int ng) { return 128 / ng; }
__host__ __device__ constexpr size_t dv_lds_bytes(int ng, int npwx_in) {
  return sizeof(cd) * 2 * (size_t)(8 * ng) * (dv_kc(ng) + 1) + sizeof(int) * (size_t)npwx_in;
}

// out(k, b, G') = scale * sum_G dvt[(m_G' - m_G) mod N] psi(k, b, G), per k the
// complex product L (G' x G) U (G x bands), L[G', G] = box(m_G' - m_G), on the
// matrix cores.  A workgroup takes four tiles of 16 rows G' (one per wave)
// and one group of 8 NG bands, and sums over G four plane waves per step.
// The 16 B columns of a band group hold the real parts of its 8 bands, then
// their imaginary parts, so that two real products per group and step (Re L
// and Im L against those columns) carry the whole complex product without
// padding bands; the two halves are combined across lanes at the end.  L
// entries are gathered from the box (L2-resident) at the row's offset plus
// the column's, the k's column offsets staged in LDS; the B values come from
// blocks of psi staged in LDS (two buffers, one barrier per block) that the
// four waves share, so that a step costs one vector load (the gather) and
// the loads of a chunk of U steps are all issued before its products.  Both
// spheres are walked in lexicographic Miller order (rows through perm_out,
// columns through perm_in, psi given in that order): the 16 rows of a tile
// and the 4 columns of a step then mostly run along z, and the 64 entries of
// a step fall on a few short runs of the box instead of 64 scattered places.
// Rows G' >= npw of the k+q sphere (the padding) are written as zero.
template <int NG>
__global__ __launch_bounds__(kDvWaves * 64) void dvpsi_mfma_kernel(
    const cd* __restrict__ box, int s2, int s3, int lo1, int lo2, int lo3, const int* __restrict__ npw_in,
    const int* __restrict__ key_in, const int* __restrict__ perm_in, int npwx_in, const cd* __restrict__ psi,
    const int* __restrict__ npw_out,
    const int* __restrict__ key_out, const int* __restrict__ perm_out, int npwx_out, cd* __restrict__ out, int nbnd,
    double scale) {
  constexpr int U = 8 / NG;
  constexpr int NB = 8 * NG;        // bands of a group
  constexpr int KC = dv_kc(NG);     // plane waves per staged block
  constexpr int BS = KC + 1;        // padded row of a staged band (bank spread)
  extern __shared__ __align__(16) char smem[];
  cd* Bs = reinterpret_cast<cd*>(smem);                    // [2][NB][BS]
  int* wcol = reinterpret_cast<int*>(Bs + 2 * NB * BS);    // [npwx_in]: -offset of m_G
  const int k = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nin = npw_in[k], nout = npw_out[k];
  for (int g = threadIdx.x; g < nin; g += kDvWaves * 64)
    wcol[g] = -miller_lin(key_in[(long)k * npwx_in + perm_in[(long)k * npwx_in + g]], s2, s3);
  __syncthreads();
  const int nbt = (nbnd + NB - 1) / NB, ngt = (npwx_out + 15) / 16, ngg = (ngt + kDvWaves - 1) / kDvWaves;
  const int l16 = lane & 15, kq = lane >> 4, part = l16 >> 3;
  const int rowoff = ((lo1 * s2) + lo2) * s3 + lo3;
  const int* pk = perm_out + (long)k * npwx_out;
  const cd* psik = psi + (long)k * nbnd * npwx_in;
  for (int wg = blockIdx.x; wg < ngg * nbt; wg += gridDim.x) {  // uniform over the workgroup
    const int gg = wg / nbt, bt = wg - gg * nbt;
    const int gt = gg * kDvWaves + wave;  // past the last tile: joins the staging, stores nothing
    // A row of this lane: the G' at position gp of the sphere in Miller
    // order; a row past the sphere reads the last one (a valid box offset),
    // its results are not stored
    const int gp = gt * 16 + l16;
    const int prow =
        nout > 0 ? miller_lin(key_out[(long)k * npwx_out + pk[gp < nout ? gp : nout - 1]], s2, s3) - rowoff : 0;
    mf64x4 d1[NG], d2[NG];
#pragma unroll
    for (int j = 0; j < NG; ++j) d1[j] = d2[j] = mf64x4{0.0, 0.0, 0.0, 0.0};
    for (int b0 = 0, buf = 0; b0 < nin && nout > 0; b0 += KC, buf ^= 1) {
      cd* bb = Bs + buf * NB * BS;
      for (int e = threadIdx.x; e < NB * KC; e += kDvWaves * 64) {
        const int bl = e / KC, g = e - bl * KC;
        const int band = bt * NB + bl;
        bb[bl * BS + g] = band < nbnd && b0 + g < nin ? psik[(long)band * npwx_in + b0 + g] : cd{0.0, 0.0};
      }
      __syncthreads();
      const double* bl[NG];
#pragma unroll
      for (int j = 0; j < NG; ++j) bl[j] = reinterpret_cast<const double*>(bb + (j * 8 + (l16 & 7)) * BS) + part;
      const int kc = min(KC, nin - b0), nfull = kc / (4 * U);
      for (int c = 0; c < nfull; ++c)
        dv_chunk_lds<NG, U, false>(box, wcol, prow, nin, b0 + c * 4 * U, b0, kq, bl, d1, d2);
      if (nfull * 4 * U < kc) dv_chunk_lds<NG, U, true>(box, wcol, prow, nin, b0 + nfull * 4 * U, b0, kq, bl, d1, d2);
    }
    // lane (kq, c), c < 8: D1 and D2 of band column c, its partner lane c + 8
    // those of the imaginary column: Re = D1[c] - D2[c + 8], Im = D1[c + 8] + D2[c]
#pragma unroll
    for (int j = 0; j < NG; ++j) {
      const int band = bt * NB + j * 8 + (l16 & 7);
      const bool colok = band < nbnd;
      cd* ob = out + ((long)k * nbnd + (colok ? band : 0)) * npwx_out;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double o1 = __shfl_xor(d1[j][r], 8, 64), o2 = __shfl_xor(d2[j][r], 8, 64);
        const int gq = gt * 16 + 4 * r + kq;  // position in Miller order; the padding maps to itself
        if (part == 0 && colok && gq < npwx_out)
          ob[pk[gq]] = gq < nout ? cd{scale * (d1[j][r] - o2), scale * (o1 + d2[j][r])} : cd{0.0, 0.0};
      }
    }
    __syncthreads();  // the next group's first block reuses buffer 0
  }
}

constexpr int kRhoWaves = 16;  // waves per workgroup of drho_mfma_kernel

// Per k: bins F_k(d) += 4 w_k M(G1, G2) over the pairs with d = m_G2 - m_G1 -
// org_k in the box [0, D1) x [0, D2) x [0, D3), for the slice x0 <= d1 < x0 +
// nx held in LDS (written to part[k]), where M = U1^H U2 (sum over the bands
// of conj(u1(G1)) u2(G2)) is formed on the matrix cores: each wave takes a
// contiguous run of 16 x 16 tiles of (G1, G2), row by row, four bands per step
// (with NBS > 0 the NBS steps of a tile row's U1 entries stay in registers
// while the row lasts, and the next tile's U2 entries are loaded while this
// tile is binned), and adds the tile's 256 values into the bins (LDS
// atomics: the order of the additions into a bin varies from run to run, so
// results agree to rounding, not bit for bit).  A bin's index is the box
// offset of m_G2 less that of m_G1 less the k's origin, from per-G offsets
// staged in LDS after the bins.  One workgroup per k; the bins fill most of a
// CU's LDS, so a workgroup is as wide as a CU takes to hide latency.
template <int NBS>
__global__ __launch_bounds__(kRhoWaves * 64) void drho_mfma_kernel(
    int nbnd, const double* __restrict__ wk, const int* __restrict__ npw1, const int* __restrict__ key1, int npwx1,
    const cd* __restrict__ u1, const int* __restrict__ npw2, const int* __restrict__ key2, int npwx2,
    const cd* __restrict__ u2, const int* __restrict__ org, int D1, int D2, int D3, int x0, int nx,
    cd* __restrict__ part) {
  extern __shared__ __align__(16) char smem[];
  const int nbin = nx * D2 * D3;
  const int nbin_al = (nbin + 1) & ~1;
  double* bre = reinterpret_cast<double*>(smem);
  double* bim = bre + nbin_al;
  int* o1s = reinterpret_cast<int*>(bim + nbin_al);  // [npwx1]
  int* o2s = o1s + npwx1;                            // [npwx2]
  const int k = blockIdx.x;
  // wave index made wave-uniform for the compiler, so that the tile walk runs
  // on the scalar unit
  const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int e = threadIdx.x; e < nbin; e += kRhoWaves * 64) bre[e] = bim[e] = 0.0;
  const int n1 = npw1[k], n2 = npw2[k];
  for (int g = threadIdx.x; g < n1; g += kRhoWaves * 64) o1s[g] = miller_lin(key1[(long)k * npwx1 + g], D2, D3);
  for (int g = threadIdx.x; g < n2; g += kRhoWaves * 64) o2s[g] = miller_lin(key2[(long)k * npwx2 + g], D2, D3);
  __syncthreads();
  const double f = 4.0 * wk[k];
  const int base = ((org[3 * k] + x0) * D2 + org[3 * k + 1]) * D3 + org[3 * k + 2];
  const int nit = (n1 + 15) / 16, njt = (n2 + 15) / 16, ntile = nit * njt;
  const int l16 = lane & 15, kq = lane >> 4;
  const int t0 = (int)((long)ntile * wave / kRhoWaves), t1 = (int)((long)ntile * (wave + 1) / kRhoWaves);
  const cd* u1k = u1 + (long)k * nbnd * npwx1;
  const cd* u2k = u2 + (long)k * nbnd * npwx2;
  constexpr int NR = NBS > 0 ? NBS : 1;
  // with the A entries in registers the weight f is folded into them
  const double fb = NBS > 0 ? 1.0 : f;
  double arc[NR], aic[NR], naic[NR], brc[NR], bic[NR];
  int o1v[4];
  // B entries of tile column jt (register path): unconditional loads from
  // clamped addresses; a band past nbnd meets a zeroed A entry, and a column
  // past the sphere is never binned
  auto fetch_b = [&](int jt) {
    const int g2 = jt * 16 + l16;
    const cd* b2 = u2k + (g2 < n2 ? g2 : 0);
#pragma unroll
    for (int s = 0; s < NR; ++s) {
      const int nu = 4 * s + kq;
      const cd b = b2[(long)(nu < nbnd ? nu : 0) * npwx2];
      brc[s] = b.x;
      bic[s] = b.y;
    }
  };
  // the wave's run of tiles is walked row by row: (it, jt) advance together
  // with t, so no tile index is divided out
  int it = t0 / njt, jt = t0 - (t0 / njt) * njt;
  int cur = -1;
  if (NBS > 0 && t0 < t1) fetch_b(jt);
  for (int t = t0; t < t1; ++t) {
    const int g1 = it * 16 + l16, g2 = jt * 16 + l16;  // this lane's A row and B column
    const bool ok1 = g1 < n1, ok2 = g2 < n2;
    int in = it, jn = jt + 1;
    if (jn == njt) {
      jn = 0;
      ++in;
    }
    mf64x4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
    if (NBS > 0) {
      if (it != cur) {
        const cd* a1 = u1k + (ok1 ? g1 : 0);
#pragma unroll
        for (int s = 0; s < NR; ++s) {
          const int nu = 4 * s + kq;
          const cd a = a1[(long)(nu < nbnd ? nu : 0) * npwx1];
          arc[s] = nu < nbnd ? f * a.x : 0.0;
          aic[s] = nu < nbnd ? -f * a.y : 0.0;  // f conj(u1); rows past the sphere are never binned
          naic[s] = -aic[s];
        }
        // box offsets of this row's G1 (rows past the sphere get a bin
        // outside the box)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int gr = it * 16 + 4 * r + kq;
          o1v[r] = gr < n1 ? o1s[gr] : INT_MIN / 2;
        }
        cur = it;
      }
#pragma unroll
      for (int s = 0; s < NR; ++s) {
        cr = mfma_16x16x4(arc[s], brc[s], cr);
        cr = mfma_16x16x4(naic[s], bic[s], cr);
        ci = mfma_16x16x4(arc[s], bic[s], ci);
        ci = mfma_16x16x4(aic[s], brc[s], ci);
      }
      // the next tile's B loads run under this tile's binning
      if (t + 1 < t1) fetch_b(jn);
    } else {
      const cd* a1 = u1k + (ok1 ? g1 : 0);
      const cd* b2 = u2k + (ok2 ? g2 : 0);
      for (int b0 = 0; b0 < nbnd; b0 += 4) {
        const int nu = b0 + kq;
        cd a = {0.0, 0.0}, b = {0.0, 0.0};
        if (nu < nbnd) {
          if (ok1) a = a1[(long)nu * npwx1];
          if (ok2) b = b2[(long)nu * npwx2];
        }
        const double ar = a.x, ai = -a.y;  // conj(u1)
        cr = mfma_16x16x4(ar, b.x, cr);
        cr = mfma_16x16x4(-ai, b.y, cr);
        ci = mfma_16x16x4(ar, b.y, ci);
        ci = mfma_16x16x4(ai, b.x, ci);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = it * 16 + 4 * r + kq;
        o1v[r] = gr < n1 ? o1s[gr] : INT_MIN / 2;
      }
    }
    // this lane's results: G1 rows 4 r + kq of the tile, G2 column l16
    if (ok2) {
      const int c2 = o2s[g2] - base;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int bin = c2 - o1v[r];
        // past the sphere, or another x-slice of the box
        if ((unsigned)bin < (unsigned)nbin) {
          atomicAdd(&bre[bin], fb * cr[r]);
          atomicAdd(&bim[bin], fb * ci[r]);
        }
      }
    }
    it = in;
    jt = jn;
  }
  __syncthreads();
  cd* dst = part + ((long)k * D1 + x0) * D2 * D3;
  for (int e = threadIdx.x; e < nbin; e += kRhoWaves * 64) dst[e] = {bre[e], bim[e]};
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
  HostStage hs(c, st);
  MKPW_TRY(hs.init(sizeof(cd) * nr, 0));
  MKPW_HIP(c, hs.up(tmp, (const cd*)dv_host, (size_t)nr));
  const dim3 grid((unsigned)((nr + 255) / 256));
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, tmp, dvt, n1, n2, n3, 0, -1, 1.0);
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, dvt, tmp, n1, n2, n3, 1, -1, 1.0);
  hipLaunchKernelGGL(mesh_dft_axis_kernel, grid, dim3(256), 0, st, tmp, dvt, n1, n2, n3, 2, -1, 1.0 / (double)nr);
  MKPW_TRY(check_launch(c, "mesh_dft", st));
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
  // the box of Miller differences m(k+q) - m(k) over every k (from each
  // sphere's Miller bounds, kept by pw_set_kpoints)
  int lo[3], sz[3];
  for (int a = 0; a < 3; ++a) {
    int dlo = 1 << 20, dhi = -(1 << 20);
    for (int k = 0; k < nk; ++k) {
      dlo = std::min(dlo, ckq->mlo[3 * k + a] - ck->mhi[3 * k + a]);
      dhi = std::max(dhi, ckq->mhi[3 * k + a] - ck->mlo[3 * k + a]);
    }
    lo[a] = dlo;
    sz[a] = std::max(1, dhi - dlo + 1);
  }
  const long nbox = (long)sz[0] * sz[1] * sz[2];
  DevBufs b(ckq);
  cd *dvt, *tmp, *W;
  MKPW_TRY(b.get((size_t)nr, &dvt));
  MKPW_TRY(b.get((size_t)nr, &tmp));
  MKPW_TRY(b.get((size_t)nk * nocc * nocc, &W));
  MKPW_TRY(transform_dv(ckq, (const double*)dv_r, dvt, tmp, st));
  // rhs0 = -dV u (on the k+q sphere)
  const int ng = nocc <= 8 ? 1 : nocc <= 16 ? 2 : 4;  // groups of 8 bands per wave
  {
    // the box of differences for all k, and psi_k with each sphere in Miller
    // order (with the k+q rows also taken in Miller order, the 64 L entries of
    // one step are a few runs of neighbours in the box)
    cd *box, *psi_sorted;
    MKPW_TRY(b.get((size_t)nbox, &box));
    MKPW_TRY(b.get((size_t)nk * nocc * ck->npwx, &psi_sorted));
    hipLaunchKernelGGL(dv_box_kernel, dim3((unsigned)((nbox + 255) / 256)), dim3(256), 0, st, dvt, ckq->fft[0],
                       ckq->fft[1], ckq->fft[2], lo[0], lo[1], lo[2], sz[0], sz[1], sz[2], box);
    hipLaunchKernelGGL(permute_rows_kernel,
                       dim3((unsigned)std::min<long>(64, ((long)nocc * ck->npwx + 255) / 256), (unsigned)nk),
                       dim3(256), 0, st, (const cd*)psi_k, ck->d_lexperm, ck->d_npw, ck->npwx, nocc, psi_sorted);
    const int ngt = (ckq->npwx + 15) / 16, nbt = (nocc + 8 * ng - 1) / (8 * ng);
    const dim3 grid((unsigned)(((ngt + kDvWaves - 1) / kDvWaves) * nbt), (unsigned)nk);
    const size_t lds = dv_lds_bytes(ng, ck->npwx);
    const void* kern = ng == 1 ? (const void*)dvpsi_mfma_kernel<1>
                       : ng == 2 ? (const void*)dvpsi_mfma_kernel<2> : (const void*)dvpsi_mfma_kernel<4>;
    MKPW_TRY(ensure_lds_limit(ckq, kern, lds));
#define MKPW_DVPSI(NG)                                                                                          \
  hipLaunchKernelGGL(dvpsi_mfma_kernel<NG>, grid, dim3(kDvWaves * 64), lds, st, box, sz[1], sz[2], lo[0], lo[1], \
                     lo[2], ck->d_npw, ck->d_mkey, ck->d_lexperm, ck->npwx, (const cd*)psi_sorted, ckq->d_npw,   \
                     ckq->d_mkey, ckq->d_lexperm, ckq->npwx, (cd*)rhs, nocc, -1.0)
    if (ng == 1) MKPW_DVPSI(1);
    else if (ng == 2) MKPW_DVPSI(2);
    else MKPW_DVPSI(4);
#undef MKPW_DVPSI
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
  // (from each sphere's Miller bounds, kept by pw_set_kpoints)
  std::vector<int> org(3 * (size_t)nk);
  int D[3] = {1, 1, 1};
  for (int k = 0; k < nk; ++k) {
    for (int a = 0; a < 3; ++a) {
      const int lo1 = ck->mlo[3 * k + a], hi1 = ck->mhi[3 * k + a];
      const int lo2 = ckq->mlo[3 * k + a], hi2 = ckq->mhi[3 * k + a];
      org[3 * k + a] = lo2 - hi1;
      D[a] = std::max(D[a], hi2 - lo1 - (lo2 - hi1) + 1);
    }
  }
  // LDS: bins of a slice of the box, then the Miller keys of both spheres
  const size_t tiles = sizeof(int) * (size_t)(ck->npwx + ckq->npwx) + 16;
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
  HostStage hs(ckq, st);
  MKPW_TRY(hs.init(sizeof(int) * org.size() + sizeof(double) * nk + 512, 0));
  MKPW_HIP(ckq, hs.up(d_org, org.data(), org.size()));
  MKPW_HIP(ckq, hs.up(d_w, wk, (size_t)nk));
  const int nbs = nbnd <= 8 ? 2 : nbnd <= 16 ? 4 : 0;  // band steps held in registers
  const void* kern = nbs == 2 ? (const void*)drho_mfma_kernel<2>
                     : nbs == 4 ? (const void*)drho_mfma_kernel<4> : (const void*)drho_mfma_kernel<0>;
  for (int x0 = 0; x0 < D[0]; x0 += nx) {
    const int nxx = std::min(nx, D[0] - x0);
    const size_t lds = per_x * nxx + tiles + 2 * sizeof(double);
    MKPW_TRY(ensure_lds_limit(ckq, kern, lds));
#define MKPW_DRHO(NBS)                                                                                             \
  hipLaunchKernelGGL(drho_mfma_kernel<NBS>, dim3((unsigned)nk), dim3(kRhoWaves * 64), lds, st, nbnd, d_w, ck->d_npw, \
                     ck->d_mkey, ck->npwx, (const cd*)psi_k, ckq->d_npw, ckq->d_mkey, ckq->npwx, (const cd*)dpsi_kq,  \
                     d_org, D[0], D[1], D[2], x0, nxx, part)
    if (nbs == 2) MKPW_DRHO(2);
    else if (nbs == 4) MKPW_DRHO(4);
    else MKPW_DRHO(0);
#undef MKPW_DRHO
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
