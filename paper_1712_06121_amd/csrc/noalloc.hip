// Allocation-free auto power spectrum: the variant of cube_get_power for callers that cannot
// allocate device memory. Its only scratch, the FP64 shell sums of Eq. (cps), lives in a
// file-scope device array of this library instead of the simulation's allocation; the outputs
// are device arrays and nothing is waited for.
#include <mutex>

#include "cube_internal.h"

namespace cube {
namespace {

constexpr int kMaxShells = 2048 / 2 + 1;  // shells 0 .. nm/2 of the largest supported mesh

// One copy per device, held until the process ends. Host code never uses this name as an address
// (it is a host-side stand-in there): kernels get the device address from hipGetSymbolAddress.
__device__ __align__(256) double scratch[3 * kMaxShells];

std::mutex g_mu;
constexpr int kMaxDevices = 64;
double* g_scratch[kMaxDevices] = {};

__global__ void k_fill_zero(double* p, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0.0;
}

// k, P and the mode count of shells 1 .. nbins from the sums (rows of nb: sum |d|^2 w, sum |n| w,
// sum w), the same FP64 operations as cube_get_power's host loop
__global__ void k_power_finish(const double* acc, int nb, int nbins, double kf, double pnorm, double* k, double* pk,
                               double* nmodes) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x + 1;
  if (b > nbins) return;
  const double w = acc[2 * nb + b];
  nmodes[b - 1] = w;
  k[b - 1] = w > 0 ? kf * acc[nb + b] / w : 0.0;
  pk[b - 1] = w > 0 ? pnorm * acc[b] / w : 0.0;
}

}  // namespace

// The device address of `scratch` on device `dev`, looked up once per device with it current.
double* noalloc_scratch(int dev) {
  if (dev < 0 || dev >= kMaxDevices) throw Error{CUBE_E_DEVICE, "device ordinal out of range"};
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    CUBE_HIP(hipGetDevice(&cur));
    if (cur != dev) CUBE_HIP(hipSetDevice(dev));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) CUBE_HIP(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      throw Error{CUBE_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
    g_scratch[dev] = static_cast<double*>(p);
  }
  return g_scratch[dev];
}

}  // namespace cube

using cube::Error;

extern "C" int cube_get_power_noalloc(cube_sim* sim, int32_t nbins, double* k, double* pk, double* nmodes) {
  if (!sim || !k || !pk || !nmodes) return CUBE_E_INVALID;
  cube::Sim& s = sim->s;
  const int nb = s.nm / 2 + 1;
  if (nbins < 1 || nbins > s.nm / 2) {
    s.last_error = "nbins must be in [1, nm/2]";
    return CUBE_E_INVALID;
  }
  if (nb > cube::kMaxShells) {
    s.last_error = "mesh too large for the fixed shell-sum array (at most " + std::to_string(cube::kMaxShells - 1) +
                   " shells)";
    return CUBE_E_INVALID;
  }
  try {
    cube::require_particles(s);
    int cur = -1;
    CUBE_HIP(hipGetDevice(&cur));
    if (cur != s.device) CUBE_HIP(hipSetDevice(s.device));
    try {
      double* acc = cube::noalloc_scratch(s.device);
      cube::launch_deposit(s, s.stream);
      // the array keeps the previous call's sums: clear this call's three rows (a kernel, so that
      // the call can be captured into a graph)
      cube::k_fill_zero<<<(3 * nb + 255) / 256, 256, 0, s.stream>>>(acc, 3 * nb);
      CUBE_HIP(hipGetLastError());
      cube::fft_power(s.mesh_plan, s.mesh, acc, s.stream);
      const double L = s.p.box, nm3 = (double)s.nm * s.nm * s.nm;
      cube::k_power_finish<<<(nbins + 255) / 256, 256, 0, s.stream>>>(acc, nb, nbins, 2.0 * M_PI / L,
                                                                        L * L * L / (nm3 * nm3), k, pk, nmodes);
      CUBE_HIP(hipGetLastError());
    } catch (...) {
      if (cur != s.device) (void)hipSetDevice(cur);
      throw;
    }
    if (cur != s.device) CUBE_HIP(hipSetDevice(cur));
  } catch (const Error& e) {
    s.last_error = e.msg;
    return e.code;
  }
  return CUBE_OK;
}
