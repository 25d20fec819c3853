// Argument types of the H|psi> kernels: the per-k tables they read and the
// selection of rows they apply H to.  Kept apart from the runtime's context so
// that the kernels' device code depends only on this file, fft.hpp, wave.hpp
// and hpsi_kernel.hpp.
#pragma once

namespace mkpw {

// Per-k tables the H|psi> kernels read (device pointers).
// The plane waves of k live in a W1 x W2 x W3 window of Miller indices
// shifted to start at 0 (m' = m - min m); a "stick" is one (m1', m2') pair
// that holds at least one plane wave.
struct KTables {
  int nk = 0, npwx = 0;
  int n1 = 0, n2 = 0, n3 = 0;
  int wx = 0, wy = 0, wz = 0;  // window extents (max over k)
  int smax = 0;                // max sticks per k
  const int* npw = nullptr;      // [nk]
  const int* nstick = nullptr;   // [nk]
  const int* gmap = nullptr;     // [nk * npwx]   (stick << 8) | m3'
  const short* sof = nullptr;    // [nk * wx * wy] stick index of (m1', m2') or -1
  const double* kin = nullptr;   // [nk * npwx]   |k+G|^2 / 2 (Ha)
};

// Which vectors to apply H to: for k, vectors [off[k], off[k] + cnt[k]) of a
// (nk, kstride) array of rows of length npwx; cnt == nullptr means all k use
// [0, nvec).
struct VecSel {
  int nvec = 0;             // grid extent in the band direction (max count)
  long kstride = 0;         // elements between consecutive k
  const int* off = nullptr; // [nk] or null
  const int* cnt = nullptr; // [nk] or null
  const int* live = nullptr;  // [nk * nvec] nonzero for rows to compute, or null (rows left unwritten)
};

}  // namespace mkpw
