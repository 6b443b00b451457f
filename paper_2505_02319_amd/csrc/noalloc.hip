// Hamiltonian application that allocates nothing: the work space of
// y = H_k x (slot and tile tables, the two column buffers of the pruned FFT,
// projector coefficients and gram partials) comes from one file-scope device
// array of fixed size instead of per-call device allocations.  For callers
// that cannot allocate device memory.
//
// Every call on one GPU shares that GPU's array (each GPU holds its own copy
// until the process ends), so calls that overlap in time on one GPU race.
// Nothing in the array has to start at zero: every entry a kernel reads is
// written earlier in the same call.
#include <mutex>

#include "system.h"

namespace ikr {

constexpr size_t SCRATCH_BYTES = size_t(64) << 20;   // 64 MiB per GPU

// The work space.  In host code `scratch` names a host-side stand-in, not
// device memory: host code only ever uses the address looked up below.
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

namespace {

constexpr int MAX_DEVICES = 64;

std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[MAX_DEVICES] = {};   // device address of scratch, per device

// Slot and tile tables of nvec vectors of k-point k (tiles of up to BT).
__global__ void ham_tables_kernel(int k, int nvec, int ntiles, int* __restrict__ sk,
                                  int* __restrict__ tk, int* __restrict__ ts,
                                  int* __restrict__ tn) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nvec) sk[i] = k;
  if (i < ntiles) {
    tk[i] = k;
    ts[i] = i * BT;
    tn[i] = min(BT, nvec - i * BT);
  }
}

}  // namespace

// Looks up the device address of the array once per device, with that
// device current (called from setup).
void init_scratch(int device) {
  IKR_CHECK(device >= 0 && device < MAX_DEVICES, IKR_E_INTERNAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return;
  void* p = nullptr;
  IKR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  IKR_CHECK(p, IKR_E_HIP, "no device address for the no-allocation work space");
  g_scratch_ptr[device] = static_cast<unsigned char*>(p);
}

void apply_hamiltonian_noalloc(System& s, int k, int nvec, const double2* x, double2* y) {
  unsigned char* base = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    base = g_scratch_ptr[s.device];
  }
  IKR_CHECK(base, IKR_E_STATE, "no-allocation work space not initialised on this device");
  const size_t need = HamWork::bytes(s, nvec);
  if (need > SCRATCH_BYTES) {
    int most = 0;
    while (most < nvec && HamWork::bytes(s, most + 1) <= SCRATCH_BYTES) ++most;
    throw Error(IKR_E_ARG, "nvec " + std::to_string(nvec) +
                               " needs " + std::to_string(need >> 20) +
                               " MiB of work space; the no-allocation limit is " +
                               std::to_string(SCRATCH_BYTES >> 20) + " MiB (" +
                               std::to_string(most) + " vectors on this system)");
  }
  HamWork w;
  w.carve(s, nvec, base);
  const int ntiles = (nvec + BT - 1) / BT;
  const int n = std::max(nvec, ntiles);
  hipLaunchKernelGGL(ham_tables_kernel, dim3((n + 255) / 256), dim3(256), 0, s.stream, k, nvec,
                     ntiles, w.sk, w.tk, w.ts, w.tn);
  IKR_HIP(hipGetLastError());
  apply_hamiltonian_ws(s, k, nvec, x, y, w);
  // a stream under graph capture cannot be synchronised: the caller's
  // replay orders the work then
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  IKR_HIP(hipStreamIsCapturing(s.stream, &cap));
  if (cap == hipStreamCaptureStatusNone) IKR_HIP(hipStreamSynchronize(s.stream));
}

}  // namespace ikr
