// Random starting vectors for the Davidson solver, drawn on the device.
//
// psi(k, b, G) = (x + i y) / (1 + |k+G|^2/2), normalised per band, where x, y
// are two N(0, 1) draws (Box-Muller) from two uniforms produced by the
// SplitMix64 finaliser (Steele, Lea & Flood 2014) chained over the counter
// (seed, k index, band, packed Miller index).  The draw at a plane wave depends
// only on that counter, so it is the same whatever the batch, the order of
// the plane waves or the device.
#include <hip/hip_runtime.h>

#include <cmath>

#include "internal.hpp"

namespace mkpw {

namespace {

__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void guess_kernel(const int* npw, int npwx, const int* mkey, const double* kin,
                                                    int nbnd, uint64_t seed, cplx<double>* psi) {
  const int k = blockIdx.y, b = blockIdx.x;
  const uint64_t key = splitmix64(splitmix64(splitmix64(seed) ^ (uint64_t)k) ^ (uint64_t)b);
  cplx<double>* row = psi + ((long)k * nbnd + b) * npwx;
  const int n = npw[k];
  __shared__ double red[4];
  double s = 0.0;
  for (int g = threadIdx.x; g < npwx; g += 256) {
    cplx<double> z = {0.0, 0.0};
    if (g < n) {
      const uint64_t h1 = splitmix64(key ^ (uint64_t)(int64_t)mkey[(long)k * npwx + g]);
      const uint64_t h2 = splitmix64(h1);
      const double u1 = 1.0 - (double)(h1 >> 11) * (1.0 / 9007199254740992.0);
      const double u2 = (double)(h2 >> 11) * (1.0 / 9007199254740992.0);
      const double r = sqrt(-2.0 * log(u1)) / (1.0 + kin[(long)k * npwx + g]);
      const double a = 2.0 * 3.14159265358979323846 * u2;
      z = {r * cos(a), r * sin(a)};
      s += z.x * z.x + z.y * z.y;
    }
    row[g] = z;
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  const double f = 1.0 / sqrt(red[0] + red[1] + red[2] + red[3]);
  for (int g = threadIdx.x; g < n; g += 256) row[g] = {row[g].x * f, row[g].y * f};
}

}  // namespace

}  // namespace mkpw

extern "C" pw_status pw_init_guess(pw_ctx* c, int nbnd, uint64_t seed, void* psi) {
  using namespace mkpw;
  if (!c) return PW_EINVAL;
  if (c->host_only) return set_err(c, PW_ESTATE, "host-only context runs no device work");
  if (!c->have_k) return set_err(c, PW_ESTATE, "set the k-points before pw_init_guess");
  if (nbnd < 1 || nbnd > 65535 || !psi) return set_err(c, PW_EINVAL, "bad nbnd or null psi");
  (void)hipSetDevice(c->device);
  hipLaunchKernelGGL(guess_kernel, dim3(nbnd, c->nk), dim3(256), 0, c->stream, c->d_npw, c->npwx, c->d_mkey, c->d_kin,
                     nbnd, seed, (cplx<double>*)psi);
  return check_launch(c, "init_guess", c->stream);
}
