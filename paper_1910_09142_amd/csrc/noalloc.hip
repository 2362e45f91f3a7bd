// Allocation-free variant of hmps_svd_probe: the truncated SVD of one
// two-site update (Chen & Stoudenmire, arXiv:1910.09142, Ancilla Method
// subsection and Results section) on caller-owned device arrays, with every
// intermediate in one file-scope device array.  For callers that cannot
// allocate device memory: no hipMalloc, no workspace, no events; the
// Jacobi sweeps are a fixed launch sequence whose rounds exit at once after
// convergence, so the only host waits are the one status read at the end.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "../../include/hmps.h"
#include "device_common.h"
#include "small_path.h"

namespace hmps {
namespace {

// Capacity: chi_l, chi_r <= NA_CHI (theta' up to 384 x 384).
constexpr int NA_CHI = 128;
constexpr int NA_MC = 3 * NA_CHI;
constexpr int NA_NCAP = npad_vectors(NA_MC);
static_assert(NA_MC < W32_MIN_N, "the rounds here are the 16-wide ones");
constexpr size_t NA_STRIDE = (size_t)((NA_MC + 15) & ~15) * NA_NCAP;
constexpr size_t NA_SITE = (size_t)3 * NA_CHI * NA_CHI;
constexpr size_t na_al(size_t doubles) { return (doubles + 31) / 32 * 32; }
constexpr int NA_QRP = (NA_MC + QB - 1) / QB;  // QR panels per stage
// layout in doubles, every piece 256-byte aligned
constexpr size_t OFF_TH = 0;
constexpr size_t OFF_X = OFF_TH + na_al(NA_STRIDE);
constexpr size_t OFF_Y = OFF_X + na_al(NA_STRIDE);
constexpr size_t OFF_Z = OFF_Y + na_al(NA_STRIDE);
constexpr size_t OFF_SITES = OFF_Z + na_al(NA_STRIDE);
constexpr size_t OFF_SIG2 = OFF_SITES + na_al(2 * NA_SITE);
constexpr size_t OFF_SIG = OFF_SIG2 + na_al(NA_NCAP);
constexpr size_t OFF_QRT = OFF_SIG + na_al(NA_NCAP);
// fac, norm2[NORM_SPLIT], logw, disc
constexpr size_t OFF_F = OFF_QRT + na_al(2 * NA_QRP * QB * QB);
constexpr size_t OFF_I = OFF_F + na_al(3 + NORM_SPLIT);  // int32 area
// int32 area (in int32 units from OFF_I): chi[3], knew, err, rot, done,
// sweeps, perm[NA_NCAP]
constexpr size_t I_CHI = 0, I_KNEW = 4, I_ERR = 5, I_ROT = 6, I_DONE = 7,
                 I_SWEEPS = 8, I_PERM = 16;
constexpr size_t NA_DOUBLES = OFF_I + na_al((I_PERM + NA_NCAP + 1) / 2);

// The scratch buffer: 5.4 MiB on every device the library runs on, held
// until the process ends and shared by every call on that device.
static __device__ __align__(256) double scratch[NA_DOUBLES];

constexpr int NA_MAX_DEVICES = 64;
std::mutex g_mutex;
double *g_ptr[NA_MAX_DEVICES] = {};

// theta (m x n row-major, device) into the vector layout of the update
// (TH and X: min(m, n) vectors of length max(m, n), stride vector_stride,
// zero padding rows), and the per-call state reset: the bond dimensions
// {chi_l, 1, chi_r} and the flags and accumulators that start at zero.
__global__ void k_na_setup(const double *theta, int chi_l, int chi_r,
                           double *base) {
  const int m = 3 * chi_l, n = 3 * chi_r;
  const bool trans = n > m;
  const int len = trans ? n : m, nvec = trans ? m : n;
  const int ld = vector_stride(len);
  double *TH = base + OFF_TH, *X = base + OFF_X;
  int32_t *iv = reinterpret_cast<int32_t *>(base + OFF_I);
  const size_t total = (size_t)ld * nvec;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int vec = (int)(e / ld), l = (int)(e % ld);
    // the vector index is interleaved (3 bond index + s)
    const int ov = (vec % 3) * (trans ? chi_l : chi_r) + vec / 3;
    double v = 0.0;
    if (l < len) v = trans ? theta[(size_t)ov * n + l] : theta[(size_t)l * n + ov];
    TH[e] = v;
    X[e] = v;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    iv[I_CHI] = chi_l;
    iv[I_CHI + 1] = 1;
    iv[I_CHI + 2] = chi_r;
    iv[I_KNEW] = 0;
    iv[I_ERR] = 0;
    iv[I_ROT] = 0;
    iv[I_DONE] = 0;
    iv[I_SWEEPS] = 0;
    for (int i = 0; i < 3 + NORM_SPLIT; ++i) base[OFF_F + i] = 0.0;
  }
}

}  // namespace
}  // namespace hmps

using namespace hmps;

extern "C" hmps_status hmps_svd_probe_noalloc(
    int32_t device, void *stream, int32_t chi_l, int32_t chi_r,
    const double *theta, int32_t chi_max, double cutoff, double *sigma,
    int32_t *rank, double *left, double *right) {
  if (!theta || !sigma || !rank || !left || !right) return HMPS_E_INVALID;
  if (chi_l < 1 || chi_r < 1 || chi_l > NA_CHI || chi_r > NA_CHI)
    return HMPS_E_INVALID;  // beyond the scratch capacity
  if (chi_max < 1 || !(cutoff >= 0.0) || !(cutoff < 1.0)) return HMPS_E_INVALID;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || device < 0 ||
      device >= n_dev || device >= NA_MAX_DEVICES)
    return HMPS_E_INVALID;
  int prev = -1;
  if (hipGetDevice(&prev) != hipSuccess) return HMPS_E_DEVICE;
  if (prev != device && hipSetDevice(device) != hipSuccess) return HMPS_E_DEVICE;
  struct Restore {
    int prev, dev;
    ~Restore() {
      if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
    }
  } restore{prev, device};
  double *base = nullptr;
  {
    // once per device, with that device current: the device address of
    // its copy of the array (in host code `scratch` names a host-side
    // stand-in, never a device address)
    std::lock_guard<std::mutex> lock(g_mutex);
    if (!g_ptr[device]) {
      void *p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
        return HMPS_E_DEVICE;
      g_ptr[device] = static_cast<double *>(p);
    }
    base = g_ptr[device];
  }
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const int m = 3 * chi_l, n = 3 * chi_r;
  const int L = m > n ? m : n, N = m > n ? n : m;
  int32_t *iv = reinterpret_cast<int32_t *>(base + OFF_I);
  Batch b;
  b.sites = base + OFF_SITES;
  b.chi = iv + I_CHI;
  b.nsites = 2;
  b.site_cap = NA_SITE;
  b.B = 1;
  UpdScratch s;
  s.TH = base + OFF_TH;
  s.X = base + OFF_X;
  s.Y = base + OFF_Y;
  s.qrT = base + OFF_QRT;
  s.qr_panels = NA_QRP;
  s.Z = base + OFF_Z;
  s.th_stride = NA_STRIDE;
  s.sig2 = base + OFF_SIG2;
  s.perm = iv + I_PERM;
  s.sig = base + OFF_SIG;
  s.n_cap = NA_NCAP;
  s.knew = iv + I_KNEW;
  s.fac = base + OFF_F;
  s.norm2 = base + OFF_F + 1;
  s.logw = base + OFF_F + 1 + NORM_SPLIT;
  s.discarded = base + OFF_F + 2 + NORM_SPLIT;
  s.rot_cur = iv + I_ROT;
  s.done = iv + I_DONE;
  s.err = iv + I_ERR;
  s.sweeps = iv + I_SWEEPS;
  s.rrk = nullptr;  // the mixed paths are never taken here
  s.rrG = nullptr;
  s.rrG_stride = 0;
  // the parameters of hmps_svd_probe on a context with chi_cap = NA_CHI
  // and default options
  UpdParams u;
  u.k = 0;
  u.gate = nullptr;
  u.is_gate = 0;
  u.right = 1;
  u.chi_max = chi_max;
  u.cutoff = cutoff;
  u.tol = 8.0 * std::sqrt(3.0 * NA_CHI) * 2.220446e-16;
  u.tol32 = 0.0;  // FP32 rounds are never launched here
  u.skip32 = 0.0;
  u.max_sweeps = 100;
  u.mixed = 0;
  u.inner_sweeps = 1;
  u.skip = 1e-30;
  u.cross_inner = 1;
  u.precond = 2;
  u.small_max = 2048;
  u.wide_min = 0;  // theta' here stays below the wide-block size
  u.zero_ok = 0;
  hipLaunchKernelGGL(k_na_setup, dim3(64), dim3(256), 0, st, theta, chi_l,
                     chi_r, base);
  if (small_path(L, N, u.small_max)) {
    launch_jacobi_small_upto(b, s, u, u.small_max, st);
  } else {
    launch_pad(b, s, u, st);
    const int path = svd_path(L, N, u.small_max, u.precond, u.mixed);
    if (path_has_qr(path)) {
      const int panels = (N + QB - 1) / QB;
      for (int stage = 0; stage < (path == PATH_QR2 ? 2 : 1); ++stage) {
        for (int p = 0; p < panels; ++p) {
          launch_qr_panel(b, s, u, stage, p, (stage == 0 ? L : N) - QB * p,
                          0, 1, st);
          launch_qr_update(b, s, u, stage, p, panels - 1 - p, 0, 1, st);
        }
        launch_qr_to_vectors(b, s, u, stage, N, 0, 1, st);
      }
    }
    // a fixed sequence of max_sweeps sweeps: once a sweep rotates nothing
    // the next sweep start marks the chain done and its rounds exit at once
    const int nb = n_blocks_even(N, JB);
    for (int sw = 0; sw < u.max_sweeps; ++sw) {
      launch_jacobi_sweep_begin(s, 1, sw, st);
      for (int r = 0; r < nb - 1; ++r)
        launch_jacobi_round(b, s, u, r, nb / 2, path_has_qr(path) ? N : L, st);
    }
    launch_jacobi_sweep_begin(s, 1, u.max_sweeps, st);
  }
  launch_truncate(b, s, u, st);
  const int kmax = std::max(1, std::min(chi_max, N));
  const bool qr2 =
      svd_path(L, N, u.small_max, u.precond, u.mixed) == PATH_QR2;
  launch_writeback(b, s, u, L, N, kmax, qr2 ? (N + QB - 1) / QB : 0, st);
  if (hipGetLastError() != hipSuccess) return HMPS_E_DEVICE;
  int32_t flags[3] = {0, 0, 0};  // knew, err, done
  if (hipMemcpyAsync(flags, iv + I_KNEW, sizeof(int32_t) * 2,
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipMemcpyAsync(flags + 2, iv + I_DONE, sizeof(int32_t),
                     hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return HMPS_E_DEVICE;
  const bool blocked = !small_path(L, N, u.small_max);
  if (flags[1] != 0 || (blocked && flags[2] == 0)) return HMPS_E_NUMERIC;
  const int k = flags[0];
  *rank = k;
  if (hipMemcpyAsync(sigma, s.sig, sizeof(double) * k,
                     hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(left, b.sites, sizeof(double) * 3 * chi_l * k,
                     hipMemcpyDeviceToDevice, st) != hipSuccess ||
      hipMemcpyAsync(right, b.sites + NA_SITE, sizeof(double) * 3 * k * chi_r,
                     hipMemcpyDeviceToDevice, st) != hipSuccess)
    return HMPS_E_DEVICE;
  return HMPS_OK;
}
