// Host runtime: context, plane-wave basis builder, FFT-mesh maps, uploads.
//
// The basis at k is every reciprocal-lattice vector G = m1 b1 + m2 b2 + m3 b3
// with |k+G|^2 < ecut_Ry (Sec. 2.2.1, sphere inequality, with E_cut in Ry and
// energies in Ha).  The FFT maps follow Sec. 4: a plane wave sits on the mesh
// at m mod N.  Because the local-potential step is a cyclic convolution on
// the mesh, translating every Miller index of one k by the same vector does
// not change its result; each k's sphere is therefore moved to start at the
// origin of its own W1 x W2 x W3 window, which lets the kernels prune the
// transforms to fixed, contiguous index ranges.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"

using namespace mkpw;

namespace mkpw {

pw_status set_err(pw_ctx* c, pw_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

pw_status dev_alloc(pw_ctx* c, size_t bytes, void** out) {
  *out = nullptr;
  if (bytes == 0) return PW_OK;
  if (c->hbm_budget > 0) {
    size_t used = 0;
    for (auto& m : c->owned) used += m.bytes;
    if ((int64_t)(used + bytes) > c->hbm_budget)
      return set_err(c, PW_ENOMEM, "HBM budget exceeded: need " + std::to_string(used + bytes) +
                                       " bytes, budget " + std::to_string(c->hbm_budget));
  }
  // stream-ordered allocation: no device-wide synchronisation, so contexts on
  // other streams (other requests) keep running while this one allocates/frees
  void* p = nullptr;
  hipError_t e = hipMallocAsync(&p, bytes, c->stream);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, PW_ENOMEM, std::string("hipMallocAsync failed: ") + hipGetErrorString(e));
  }
  c->owned.push_back({p, bytes});
  *out = p;
  return PW_OK;
}

pw_status host_pinned(pw_ctx* c, size_t bytes, void** out) {
  // copies queued by an earlier call that ended early may still read the
  // buffer: they finish before it is reused or replaced
  hipError_t e = hipStreamSynchronize(c->stream);
  if (e == hipSuccess && bytes > c->pin_cap) {
    if (c->pin) (void)hipHostFree(c->pin);
    c->pin = nullptr;
    c->pin_cap = 0;
    const size_t cap = std::max(bytes, (size_t)1 << 16);
    e = hipHostMalloc(&c->pin, cap, hipHostMallocDefault);
    if (e == hipSuccess) c->pin_cap = cap;
  }
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, PW_EDEVICE, std::string("page-locked staging: ") + hipGetErrorString(e));
  }
  *out = c->pin;
  return PW_OK;
}

void dev_free(pw_ctx* c, void* p) {
  if (!p) return;
  for (size_t i = 0; i < c->owned.size(); ++i) {
    if (c->owned[i].p == p) {
      (void)hipFreeAsync(p, c->stream);
      c->owned.erase(c->owned.begin() + i);
      return;
    }
  }
}

// Every query or change of a kernel's attributes in the process goes through
// this lock: contexts on several host threads tune and launch at once.
std::mutex g_attr_mu;
std::unordered_map<const void*, size_t> g_lds_limit;                  // dynamic LDS allowed per kernel
std::unordered_map<const void*, std::pair<int, size_t>> g_resources;  // registers, scratch bytes per lane

bool kernel_resources(const void* kernel, int* regs, size_t* scratch) {
  std::lock_guard<std::mutex> lk(g_attr_mu);
  auto it = g_resources.find(kernel);
  if (it == g_resources.end()) {
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, kernel) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    it = g_resources.emplace(kernel, std::make_pair(a.numRegs, a.localSizeBytes)).first;
  }
  *regs = it->second.first;
  *scratch = it->second.second;
  return true;
}

pw_status ensure_lds_limit(pw_ctx* c, const void* kernel, size_t lds) {
  // Raise a kernel's dynamic-LDS limit to the CU's 160 KiB once per process,
  // under the attribute lock and before the first launch of that kernel, so
  // that no thread changes a kernel's attributes while another thread
  // launches it or reads them.
  if (lds <= 64 * 1024) return PW_OK;
  std::lock_guard<std::mutex> lk(g_attr_mu);
  auto& limit = g_lds_limit;
  auto it = limit.find(kernel);
  if (it == limit.end()) {
    hipFuncAttributes fa;
    hipError_t e = hipFuncGetAttributes(&fa, kernel);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_err(c, PW_EDEVICE, std::string("hipFuncGetAttributes: ") + hipGetErrorString(e));
    }
    const size_t dyn_max = 160 * 1024 - fa.sharedSizeBytes;  // the CU's LDS minus the kernel's static LDS
    e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_max);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      return set_err(c, PW_EDEVICE, std::string("hipFuncSetAttribute: ") + hipGetErrorString(e));
    }
    it = limit.emplace(kernel, dyn_max).first;
  }
  if (lds > it->second) return set_err(c, PW_EINVAL, "kernel LDS request above what a CU provides");
  return PW_OK;
}

}  // namespace mkpw

mkpw::KTables pw_ctx::tables() const {
  KTables t;
  t.nk = nk;
  t.npwx = npwx;
  t.n1 = fft[0];
  t.n2 = fft[1];
  t.n3 = fft[2];
  t.wx = wx;
  t.wy = wy;
  t.wz = wz;
  t.smax = smax;
  t.npw = d_npw;
  t.nstick = d_nstick;
  t.gmap = d_gmap;
  t.sof = d_sof;
  t.kin = d_kin;
  return t;
}

namespace {

#define HIPCHK(c, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      (void)hipGetLastError();                                                           \
      return set_err((c), PW_EDEVICE, std::string(#call " failed: ") + hipGetErrorString(e_)); \
    }                                                                                    \
  } while (0)

void clear_q(pw_ctx* c) {
  for (void** p : {&c->d_q64, &c->d_q32}) {
    dev_free(c, *p);
    *p = nullptr;
  }
  c->have_q = false;
  c->qij.clear();
}

void free_kdata(pw_ctx* c) {
  for (void** p : {(void**)&c->d_npw, (void**)&c->d_nstick, (void**)&c->d_gmap, (void**)&c->d_sof,
                   (void**)&c->d_kin, (void**)&c->d_mkey, (void**)&c->d_lexperm, (void**)&c->d_beta64,
                   (void**)&c->d_beta32}) {
    dev_free(c, *p);
    *p = nullptr;
  }
  c->have_k = false;
  c->have_proj = false;
  c->nproj = 0;
  clear_q(c);
}

void free_all(pw_ctx* c) {
  free_kdata(c);
  for (void** p : {(void**)&c->d_v64, (void**)&c->d_v32, (void**)&c->d_dij64, (void**)&c->d_dij32,
                   (void**)&c->d_vperm64, (void**)&c->d_vperm32, (void**)&c->d_xtaps64, (void**)&c->d_xtaps32}) {
    dev_free(c, *p);
    *p = nullptr;
  }
  c->vperm_l3c64 = c->vperm_l3c32 = 0;
  c->xtaps_wc64 = c->xtaps_wc32 = 0;
  c->have_v = false;
}

int smooth235(int n) {
  for (;; ++n) {
    int m = n;
    for (int p : {2, 3, 5})
      while (m % p == 0) m /= p;
    if (m == 1) return n;
  }
}

// projector rows as uploaded: zero the padding (g >= npw[k]) so kernels may
// read whole rows, and form the complex64 copy
__global__ void prepare_beta_kernel(double* b64, float* b32, const int* npw, int nproj, int npwx, long nrows) {
  const long total = nrows * npwx;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const long row = e / npwx;
    const int g = (int)(e - row * npwx), k = (int)(row / nproj);
    double re = b64[2 * e], im = b64[2 * e + 1];
    if (g >= npw[k]) {
      re = im = 0.0;
      b64[2 * e] = b64[2 * e + 1] = 0.0;
    }
    b32[2 * e] = (float)re;
    b32[2 * e + 1] = (float)im;
  }
}

template <class T>
pw_status upload(pw_ctx* c, const T* host, size_t count, T** dev) {
  void* p = nullptr;
  pw_status s = dev_alloc(c, count * sizeof(T), &p);
  if (s != PW_OK) return s;
  *dev = (T*)p;
  if (count) HIPCHK(c, hipMemcpyAsync(p, host, count * sizeof(T), hipMemcpyHostToDevice, c->stream));
  return PW_OK;
}

}  // namespace

extern "C" {

namespace {
// The solvers' work buffers are stream-ordered allocations from the device's
// default memory pool.  With the pool's default release threshold (0) its
// memory goes back to the system at every synchronisation, so each call maps
// its buffers anew; keeping up to an eighth of the device (at most 32 GiB)
// cached lets repeated calls reuse them.  Set once per device and process.
void keep_pool_memory(int device) {
  static std::mutex mu;
  static std::vector<int> done;
  std::lock_guard<std::mutex> lk(mu);
  if (std::find(done.begin(), done.end(), device) != done.end()) return;
  done.push_back(device);
  hipMemPool_t pool = nullptr;
  size_t free_b = 0, total_b = 0;
  if (hipDeviceGetDefaultMemPool(&pool, device) != hipSuccess || hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
    (void)hipGetLastError();
    return;
  }
  uint64_t keep = std::min<uint64_t>((uint64_t)total_b / 8, (uint64_t)32 << 30);
  if (hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep) != hipSuccess) (void)hipGetLastError();
}
}  // namespace

pw_status pw_create(pw_ctx** out, int hip_device, void* hip_stream) {
  if (!out) return PW_EINVAL;
  *out = nullptr;
  pw_ctx* c = new (std::nothrow) pw_ctx();
  if (!c) return PW_ENOMEM;
  c->device = hip_device;
  c->host_only = hip_device < 0;
  if (!c->host_only) {
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || hip_device >= n) {
      (void)hipGetLastError();
      delete c;
      return PW_EDEVICE;
    }
    if (hipSetDevice(hip_device) != hipSuccess) {
      delete c;
      return PW_EDEVICE;
    }
    keep_pool_memory(hip_device);
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return PW_EDEVICE;
      }
      c->own_stream = true;
    }
    // this device's copy of the staging array of pw_h_psi_noalloc
    if (mkpw::hpsi_scratch_init(c) != PW_OK) {
      if (c->own_stream) (void)hipStreamDestroy(c->stream);
      delete c;
      return PW_EDEVICE;
    }
  }
  *out = c;
  return PW_OK;
}

void pw_destroy(pw_ctx* c) {
  if (!c) return;
  if (!c->host_only) {
    (void)hipSetDevice(c->device);
    for (auto& m : c->owned) (void)hipFreeAsync(m.p, c->stream);
    c->owned.clear();
    (void)hipStreamSynchronize(c->stream);
    if (c->pin) (void)hipHostFree(c->pin);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
  }
  delete c;
}

const char* pw_last_error(const pw_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

pw_status pw_set_option(pw_ctx* c, const char* key, int64_t value) {
  if (!c || !key) return PW_EINVAL;
  std::string k(key);
  if (k == "hbm_budget_bytes") {
    if (value < 0) return set_err(c, PW_EINVAL, "hbm_budget_bytes must be >= 0");
    c->hbm_budget = value;
  } else if (k == "davidson_basis_factor") {
    if (value < 2 || value > 16) return set_err(c, PW_EINVAL, "davidson_basis_factor must be in [2, 16]");
    c->dav_basis_factor = value;
  } else if (k == "trace") {
    c->trace = value;
  } else if (k == "hpsi_variant") {
    if (value < 0 || value > 5) return set_err(c, PW_EINVAL, "hpsi_variant must be in [0, 5]");
    c->hpsi_variant = value;
  } else if (k == "hpsi_slab") {
    if (value < 0 || value > 512) return set_err(c, PW_EINVAL, "hpsi_slab must be in [0, 512]");
    c->hpsi_slab = value;
  } else if (k == "hpsi_threads") {
    if (value != 0 && value != 256 && value != 512 && value != 1024)
      return set_err(c, PW_EINVAL, "hpsi_threads must be 0, 256, 512 or 1024");
    c->hpsi_threads = value;
  } else if (k == "tune_log") {
    c->tune_log = value;
  } else if (k == "solver_graph") {
    c->solver_graph = value != 0;
  } else if (k == "mixed_refine") {
    c->mixed_refine = value != 0;
  } else if (k == "mixed_switch_rtol_e7") {
    if (value < 100 || value > 100000) return set_err(c, PW_EINVAL, "mixed_switch_rtol_e7 must be in [100, 100000]");
    c->mixed_switch_rtol_e7 = value;
  } else if (k == "dav_nconv") {
    if (value < 0 || value > 1024) return set_err(c, PW_EINVAL, "dav_nconv must be in [0, 1024]");
    c->dav_nconv = value;
  } else if (k == "cg_switch_digits") {
    if (value < 2 || value > 20) return set_err(c, PW_EINVAL, "cg_switch_digits must be in [2, 20]");
    c->cg_switch_digits = value;
  } else {
    return set_err(c, PW_EINVAL, "unknown option '" + k + "'");
  }
  return PW_OK;
}

pw_status pw_get_option(const pw_ctx* c, const char* key, int64_t* value) {
  if (!c || !key || !value) return PW_EINVAL;
  std::string k(key);
  if (k == "hbm_budget_bytes") *value = c->hbm_budget;
  else if (k == "davidson_basis_factor") *value = c->dav_basis_factor;
  else if (k == "trace") *value = c->trace;
  else if (k == "hpsi_variant") *value = c->hpsi_variant;
  else if (k == "hpsi_slab") *value = c->hpsi_slab;
  else if (k == "hpsi_variant_tuned") *value = c->last_hpsi_variant;
  else if (k == "hpsi_threads") *value = c->hpsi_threads;
  else if (k == "hpsi_slab_tuned") *value = c->last_hpsi_slab;
  else if (k == "hpsi_threads_tuned") *value = c->last_hpsi_threads;
  else if (k == "tune_log") *value = c->tune_log;
  else if (k == "solver_graph") *value = c->solver_graph;
  else if (k == "mixed_refine") *value = c->mixed_refine;
  else if (k == "mixed_switch_rtol_e7") *value = c->mixed_switch_rtol_e7;
  else if (k == "cg_switch_digits") *value = c->cg_switch_digits;
  else if (k == "dav_nconv") *value = c->dav_nconv;
  else if (k == "last_iterations") *value = c->last_iterations;
  else if (k == "last_hpsi_kbands") *value = c->last_hpsi_kbands;
  else if (k == "last_graph_replays") *value = c->last_graph_replays;
  else if (k == "overlap") *value = c->have_q ? 1 : 0;
  else if (k == "nk") *value = c->have_k ? c->nk : 0;
  else if (k == "npwx") *value = c->have_k ? c->npwx : 0;
  else if (k == "nproj") *value = c->have_proj ? c->nproj : 0;
  else if (k == "fft1" || k == "fft2" || k == "fft3") *value = c->have_cutoff ? c->fft[k[3] - '1'] : 0;
  else if (k == "device_bytes") {
    int64_t b = 0;
    for (auto& m : c->owned) b += (int64_t)m.bytes;
    *value = b;
  } else {
    return set_err(const_cast<pw_ctx*>(c), PW_EINVAL, "unknown option '" + k + "'");
  }
  return PW_OK;
}

pw_status pw_set_lattice(pw_ctx* c, const double a[9]) {
  if (!c || !a) return PW_EINVAL;
  double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
               a[2] * (a[3] * a[7] - a[4] * a[6]);
  if (!(std::fabs(det) > 1e-8)) return set_err(c, PW_EINVAL, "lattice vectors are singular");
  if (!c->host_only) (void)hipSetDevice(c->device);
  free_all(c);
  std::memcpy(c->lat, a, sizeof(c->lat));
  // b_j = 2 pi (a_k x a_l) / det  so that a_i . b_j = 2 pi delta_ij
  const double* a1 = a;
  const double* a2 = a + 3;
  const double* a3 = a + 6;
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double t[3];
  const double f = 2.0 * M_PI / det;
  cross(a2, a3, t);
  for (int i = 0; i < 3; ++i) c->rec[0 + i] = f * t[i];
  cross(a3, a1, t);
  for (int i = 0; i < 3; ++i) c->rec[3 + i] = f * t[i];
  cross(a1, a2, t);
  for (int i = 0; i < 3; ++i) c->rec[6 + i] = f * t[i];
  c->have_lattice = true;
  c->have_cutoff = false;
  c->have_k = false;
  return PW_OK;
}

pw_status pw_set_cutoff(pw_ctx* c, double ecut, const int fft[3]) {
  if (!c || !fft) return PW_EINVAL;
  if (!c->have_lattice) return set_err(c, PW_ESTATE, "set the lattice before the cutoff");
  if (!(ecut > 0) || ecut > 1e4) return set_err(c, PW_EINVAL, "cutoff must be in (0, 1e4] Ry");
  int n[3];
  for (int i = 0; i < 3; ++i) {
    if (fft[i] < 0 || fft[i] > 512) return set_err(c, PW_EINVAL, "FFT mesh dimension out of range");
    if (fft[i] == 0) {
      const double* ai = c->lat + 3 * i;
      double na = std::sqrt(ai[0] * ai[0] + ai[1] * ai[1] + ai[2] * ai[2]);
      n[i] = smooth235(2 * (int)std::floor(2.0 * std::sqrt(ecut) * na / (2.0 * M_PI)) + 1);
    } else {
      n[i] = fft[i];
    }
  }
  if ((fft[0] == 0) != (fft[1] == 0) || (fft[0] == 0) != (fft[2] == 0))
    return set_err(c, PW_EINVAL, "FFT mesh: give all three dimensions or none");
  if (!c->host_only) (void)hipSetDevice(c->device);
  free_all(c);
  c->ecut_ry = ecut;
  std::memcpy(c->fft, n, sizeof(n));
  c->have_cutoff = true;
  return PW_OK;
}

pw_status pw_set_kpoints(pw_ctx* c, int nk, const double* k, int32_t* npw_out, int32_t* npwx_out) {
  if (!c || (nk > 0 && !k)) return PW_EINVAL;
  if (!c->have_cutoff) return set_err(c, PW_ESTATE, "set lattice and cutoff before the k-points");
  if (nk <= 0 || nk > (1 << 22)) return set_err(c, PW_EINVAL, "nk must be in [1, 2^22]");
  if (!c->host_only) (void)hipSetDevice(c->device);
  free_kdata(c);
  const double* b = c->rec;
  const double kc = std::sqrt(c->ecut_ry);
  struct PW {
    double q2;
    int m[3];
    int gen;  // position in the lexicographic (m1, m2, m3) enumeration
  };
  std::vector<std::vector<PW>> all(nk);
  std::vector<std::vector<int>> lexpos(nk);  // per k: sorted position of the j-th G in Miller order
  // spheres of the k-points built and sorted in parallel host threads, each
  // over its own range of k
  auto build_range = [&](int k0, int k1) {
  for (int ik = k0; ik < k1; ++ik) {
    const double* kk = k + 3 * ik;
    int lo[3], hi[3];
    for (int i = 0; i < 3; ++i) {
      const double* ai = c->lat + 3 * i;
      double na = std::sqrt(ai[0] * ai[0] + ai[1] * ai[1] + ai[2] * ai[2]);
      double kd = (kk[0] * ai[0] + kk[1] * ai[1] + kk[2] * ai[2]) / (2.0 * M_PI);
      double r = kc * na / (2.0 * M_PI);
      lo[i] = (int)std::floor(-kd - r) - 1;
      hi[i] = (int)std::ceil(-kd + r) + 1;
    }
    auto& v = all[ik];
    for (int m1 = lo[0]; m1 <= hi[0]; ++m1)
      for (int m2 = lo[1]; m2 <= hi[1]; ++m2)
        for (int m3 = lo[2]; m3 <= hi[2]; ++m3) {
          double q[3];
          for (int d = 0; d < 3; ++d) q[d] = kk[d] + m1 * b[d] + m2 * b[3 + d] + m3 * b[6 + d];
          double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
          if (q2 < c->ecut_ry) v.push_back({q2, {m1, m2, m3}, (int)v.size()});
        }
    std::sort(v.begin(), v.end(), [](const PW& x, const PW& y) {
      if (x.q2 != y.q2) return x.q2 < y.q2;
      return std::lexicographical_compare(x.m, x.m + 3, y.m, y.m + 3);
    });
    auto& lp = lexpos[ik];
    lp.resize(v.size());
    for (size_t i = 0; i < v.size(); ++i) lp[v[i].gen] = (int)i;
  }
  };
  {
    const int hw = std::max(1u, std::thread::hardware_concurrency());
    const int nt = std::max(1, std::min({hw, 16, nk / 16}));
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(build_range, (int)((long)nk * t / nt), (int)((long)nk * (t + 1) / nt));
    build_range(0, (int)((long)nk / nt));
    for (auto& x : th) x.join();
  }
  int npwmax = 0;
  for (int ik = 0; ik < nk; ++ik) npwmax = std::max<int>(npwmax, (int)all[ik].size());
  if (npwmax == 0) return set_err(c, PW_EINVAL, "empty plane-wave basis");
  const int npwx = (npwmax + 63) / 64 * 64;

  // window of every k (Miller indices shifted to start at 0) and the global extents
  std::vector<std::array<int, 3>> lo(nk);
  int wmax[3] = {0, 0, 0};
  for (int ik = 0; ik < nk; ++ik) {
    int mn[3] = {1 << 30, 1 << 30, 1 << 30}, mx[3] = {-(1 << 30), -(1 << 30), -(1 << 30)};
    for (auto& p : all[ik])
      for (int d = 0; d < 3; ++d) {
        mn[d] = std::min(mn[d], p.m[d]);
        mx[d] = std::max(mx[d], p.m[d]);
      }
    if (all[ik].empty())
      for (int d = 0; d < 3; ++d) mn[d] = mx[d] = 0;
    for (int d = 0; d < 3; ++d) {
      lo[ik][d] = mn[d];
      wmax[d] = std::max(wmax[d], mx[d] - mn[d] + 1);
    }
  }
  c->mlo.assign((size_t)3 * nk, 0);
  c->mhi.assign((size_t)3 * nk, 0);
  for (int ik = 0; ik < nk; ++ik)
    for (int d = 0; d < 3; ++d) {
      int mx = lo[ik][d];
      for (auto& p : all[ik]) mx = std::max(mx, p.m[d]);
      c->mlo[3 * ik + d] = lo[ik][d];
      c->mhi[3 * ik + d] = mx;
    }
  for (int d = 0; d < 3; ++d)
    if (wmax[d] > c->fft[d])
      return set_err(c, PW_EINVAL,
                     "FFT mesh too small: the plane-wave sphere spans " + std::to_string(wmax[d]) +
                         " points along axis " + std::to_string(d + 1) + " but N = " + std::to_string(c->fft[d]));
  if (wmax[2] > 255) return set_err(c, PW_EINVAL, "sphere too wide along axis 3");
  for (int ik = 0; ik < nk; ++ik)
    for (auto& p : all[ik])
      for (int d = 0; d < 3; ++d)
        if (p.m[d] < -512 || p.m[d] > 511) return set_err(c, PW_EINVAL, "Miller index outside [-512, 511]");

  const int wx = wmax[0], wy = wmax[1], wz = wmax[2];
  c->nk = nk;
  c->npwx = npwx;
  c->wx = wx;
  c->wy = wy;
  c->wz = wz;
  c->kcart.assign(k, k + 3 * nk);
  c->npw.assign(nk, 0);
  c->nstick.assign(nk, 0);
  c->miller.assign((size_t)nk * npwx * 3, 0);
  c->kin.assign((size_t)nk * npwx, 0.0);
  c->gmap.assign((size_t)nk * npwx, 0);
  c->sof.assign((size_t)nk * wx * wy, (short)-1);
  int smax = 0;
  for (int ik = 0; ik < nk; ++ik) {
    auto& v = all[ik];
    int n = (int)v.size();
    c->npw[ik] = n;
    short* sof = c->sof.data() + (size_t)ik * wx * wy;
    for (auto& p : v) sof[(p.m[0] - lo[ik][0]) * wy + (p.m[1] - lo[ik][1])] = 0;
    int ns = 0;
    for (int i = 0; i < wx * wy; ++i)
      if (sof[i] == 0) sof[i] = (short)ns++;
      else sof[i] = -1;
    if (ns > 32767) return set_err(c, PW_EINVAL, "too many FFT sticks");
    c->nstick[ik] = ns;
    smax = std::max(smax, ns);
    for (int g = 0; g < n; ++g) {
      const auto& p = v[g];
      size_t o = (size_t)ik * npwx + g;
      for (int d = 0; d < 3; ++d) c->miller[o * 3 + d] = p.m[d];
      c->kin[o] = 0.5 * p.q2;
      int s = sof[(p.m[0] - lo[ik][0]) * wy + (p.m[1] - lo[ik][1])];
      c->gmap[o] = (s << 8) | (p.m[2] - lo[ik][2]);
    }
  }
  c->smax = smax;
  if (npw_out)
    for (int ik = 0; ik < nk; ++ik) npw_out[ik] = c->npw[ik];
  if (npwx_out) *npwx_out = npwx;

  if (!c->host_only) {
    pw_status s;
    if ((s = upload(c, c->npw.data(), c->npw.size(), &c->d_npw)) != PW_OK) return s;
    if ((s = upload(c, c->nstick.data(), c->nstick.size(), &c->d_nstick)) != PW_OK) return s;
    if ((s = upload(c, c->gmap.data(), c->gmap.size(), &c->d_gmap)) != PW_OK) return s;
    if ((s = upload(c, c->sof.data(), c->sof.size(), &c->d_sof)) != PW_OK) return s;
    if ((s = upload(c, c->kin.data(), c->kin.size(), &c->d_kin)) != PW_OK) return s;
    std::vector<int> mkey((size_t)nk * npwx, 0);
    for (size_t o = 0; o < mkey.size(); ++o) {
      const int32_t* m = c->miller.data() + 3 * o;
      mkey[o] = ((m[0] + 512) << 20) | ((m[1] + 512) << 10) | (m[2] + 512);
    }
    if ((s = upload(c, mkey.data(), mkey.size(), &c->d_mkey)) != PW_OK) return s;
    // each sphere in lexicographic Miller order (m3 fastest, the order the
    // spheres were enumerated in); the padding maps to itself
    std::vector<int> lex((size_t)nk * npwx);
    for (int ik = 0; ik < nk; ++ik) {
      int* p = lex.data() + (size_t)ik * npwx;
      const int n = c->npw[ik];
      std::copy(lexpos[ik].begin(), lexpos[ik].end(), p);
      for (int i = n; i < npwx; ++i) p[i] = i;
    }
    if ((s = upload(c, lex.data(), lex.size(), &c->d_lexperm)) != PW_OK) return s;
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->have_k = true;
  return PW_OK;
}

pw_status pw_get_miller(const pw_ctx* c, int ik, int32_t* miller) {
  if (!c || !miller) return PW_EINVAL;
  if (!c->have_k) return set_err(const_cast<pw_ctx*>(c), PW_ESTATE, "no k-points set");
  if (ik == -1) {  // every k, concatenated
    size_t o = 0;
    for (int k = 0; k < c->nk; ++k) {
      std::memcpy(miller + o, c->miller.data() + (size_t)k * c->npwx * 3, sizeof(int32_t) * 3 * c->npw[k]);
      o += 3 * (size_t)c->npw[k];
    }
    return PW_OK;
  }
  if (ik < 0 || ik >= c->nk) return set_err(const_cast<pw_ctx*>(c), PW_EINVAL, "k index out of range");
  std::memcpy(miller, c->miller.data() + (size_t)ik * c->npwx * 3, sizeof(int32_t) * 3 * c->npw[ik]);
  return PW_OK;
}

pw_status pw_set_vloc(pw_ctx* c, const double* v) {
  if (!c || !v) return PW_EINVAL;
  if (!c->have_cutoff) return set_err(c, PW_ESTATE, "set lattice and cutoff before the potential");
  const size_t nr = (size_t)c->fft[0] * c->fft[1] * c->fft[2];
  for (size_t i = 0; i < nr; ++i)
    if (!std::isfinite(v[i])) return set_err(c, PW_EINVAL, "potential has a non-finite value");
  if (c->host_only) {
    c->have_v = true;
    return PW_OK;
  }
  (void)hipSetDevice(c->device);
  // the forward transform's 1/N_r (Eq. fwFFT) is folded into the potential
  std::vector<double> v64(nr);
  std::vector<float> v32(nr);
  double vsum = 0.0;
  for (size_t i = 0; i < nr; ++i) vsum += v[i];
  c->v0 = vsum / (double)nr;
  for (size_t i = 0; i < nr; ++i) {
    v64[i] = v[i] / (double)nr;
    v32[i] = (float)v64[i];
  }
  dev_free(c, c->d_v64);
  dev_free(c, c->d_v32);
  c->d_v64 = nullptr;
  c->d_v32 = nullptr;
  c->vperm_l3c64 = c->vperm_l3c32 = 0;  // permuted copies and x taps are rebuilt from the new potential
  c->xtaps_wc64 = c->xtaps_wc32 = 0;
  c->have_v = false;
  pw_status s;
  if ((s = upload(c, v64.data(), nr, &c->d_v64)) != PW_OK) return s;
  if ((s = upload(c, v32.data(), nr, &c->d_v32)) != PW_OK) return s;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->have_v = true;
  return PW_OK;
}

pw_status pw_set_projectors(pw_ctx* c, int nproj, const void* beta, const void* dij) {
  if (!c) return PW_EINVAL;
  if (!c->have_k) return set_err(c, PW_ESTATE, "set the k-points before the projectors");
  if (nproj < 0 || nproj > 32) return set_err(c, PW_EINVAL, "nproj must be in [0, 32]");
  if (nproj > 0 && (!beta || !dij)) return set_err(c, PW_EINVAL, "null projector or D array");
  const double* d = (const double*)dij;
  double dmax = 0.0, herm = 0.0;
  for (int p = 0; p < nproj; ++p)
    for (int q = 0; q < nproj; ++q) {
      double re = d[2 * (p * nproj + q)], im = d[2 * (p * nproj + q) + 1];
      double rt = d[2 * (q * nproj + p)], it = d[2 * (q * nproj + p) + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) return set_err(c, PW_EINVAL, "D has a non-finite value");
      dmax = std::max(dmax, std::hypot(re, im));
      herm = std::max(herm, std::hypot(re - rt, im + it));
    }
  if (herm > 1e-12 * std::max(dmax, 1e-300) && herm > 0)
    return set_err(c, PW_EINVAL, "D is not Hermitian");
  const size_t nb = (size_t)c->nk * nproj * c->npwx;
  const double* bsrc = (const double*)beta;
  for (size_t i = 0; i < 2 * nb; ++i)
    if (!std::isfinite(bsrc[i])) return set_err(c, PW_EINVAL, "projector array has a non-finite value");
  c->dij.assign(d, d + 2 * (size_t)nproj * nproj);
  clear_q(c);
  if (c->host_only) {
    c->nproj = nproj;
    c->have_proj = true;
    return PW_OK;
  }
  (void)hipSetDevice(c->device);
  for (void** p : {(void**)&c->d_beta64, (void**)&c->d_beta32, (void**)&c->d_dij64, (void**)&c->d_dij32}) {
    dev_free(c, *p);
    *p = nullptr;
  }
  c->have_proj = false;
  c->nproj = 0;
  if (nproj > 0) {
    // rows uploaded as given; the padding is zeroed and the complex64 copy
    // formed on the device
    std::vector<float> d32(2 * (size_t)nproj * nproj);
    for (size_t i = 0; i < d32.size(); ++i) d32[i] = (float)d[i];
    pw_status s;
    double* p64 = nullptr;
    float* p32 = nullptr;
    if ((s = upload(c, bsrc, 2 * nb, &p64)) != PW_OK) return s;
    c->d_beta64 = p64;
    void* v32 = nullptr;
    if ((s = dev_alloc(c, 2 * nb * sizeof(float), &v32)) != PW_OK) return s;
    c->d_beta32 = v32;
    hipLaunchKernelGGL(prepare_beta_kernel, dim3(1024), dim3(256), 0, c->stream, p64, (float*)v32, c->d_npw, nproj,
                       c->npwx, (long)c->nk * nproj);
    HIPCHK(c, hipGetLastError());
    if ((s = upload(c, d, 2 * (size_t)nproj * nproj, &p64)) != PW_OK) return s;
    c->d_dij64 = p64;
    if ((s = upload(c, d32.data(), d32.size(), &p32)) != PW_OK) return s;
    c->d_dij32 = p32;
    HIPCHK(c, hipStreamSynchronize(c->stream));
  }
  c->nproj = nproj;
  c->have_proj = true;
  return PW_OK;
}

pw_status pw_set_qij(pw_ctx* c, const void* qij) {
  if (!c) return PW_EINVAL;
  if (!qij) {
    clear_q(c);
    return PW_OK;
  }
  if (!c->have_proj || c->nproj == 0) return set_err(c, PW_ESTATE, "set projectors (nproj > 0) before q");
  const int n = c->nproj;
  const double* q = (const double*)qij;
  double qmax = 0.0, herm = 0.0;
  for (int p = 0; p < n; ++p)
    for (int r = 0; r < n; ++r) {
      double re = q[2 * (p * n + r)], im = q[2 * (p * n + r) + 1];
      double rt = q[2 * (r * n + p)], it = q[2 * (r * n + p) + 1];
      if (!std::isfinite(re) || !std::isfinite(im)) return set_err(c, PW_EINVAL, "q has a non-finite value");
      qmax = std::max(qmax, std::hypot(re, im));
      herm = std::max(herm, std::hypot(re - rt, im + it));
    }
  if (herm > 1e-12 * std::max(qmax, 1e-300) && herm > 0) return set_err(c, PW_EINVAL, "q is not Hermitian");
  clear_q(c);
  c->qij.assign(q, q + 2 * (size_t)n * n);
  if (c->host_only) {
    c->have_q = true;
    return PW_OK;
  }
  (void)hipSetDevice(c->device);
  std::vector<float> q32(2 * (size_t)n * n);
  for (size_t i = 0; i < q32.size(); ++i) q32[i] = (float)q[i];
  pw_status s;
  double* p64 = nullptr;
  float* p32 = nullptr;
  if ((s = upload(c, q, 2 * (size_t)n * n, &p64)) != PW_OK) return s;
  c->d_q64 = p64;
  if ((s = upload(c, q32.data(), q32.size(), &p32)) != PW_OK) return s;
  c->d_q32 = p32;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  c->have_q = true;
  return PW_OK;
}

pw_status pw_h_psi(pw_ctx* c, pw_prec prec, int nbnd, const void* psi, void* hpsi) {
  if (!c) return PW_EINVAL;
  if (c->host_only) return set_err(c, PW_ESTATE, "host-only context runs no device work");
  if (!c->have_k || !c->have_v) return set_err(c, PW_ESTATE, "set k-points and potential before h_psi");
  if (prec != PW_FP64 && prec != PW_MIXED) return set_err(c, PW_EINVAL, "unknown precision");
  if (nbnd <= 0 || nbnd > 65535) return set_err(c, PW_EINVAL, "nbnd must be in [1, 65535]");
  if (!psi || !hpsi) return set_err(c, PW_EINVAL, "null psi or hpsi");
  (void)hipSetDevice(c->device);
  VecSel sel;
  sel.nvec = nbnd;
  sel.kstride = (long)nbnd * c->npwx;
  return launch_hpsi(c, prec, sel, psi, hpsi, c->stream);
}

}  // extern "C"
