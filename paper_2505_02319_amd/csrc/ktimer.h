// Opt-in per-kernel timing with HIP events on the launching stream.
// When enabled, begin()/end() bracket a launch with two events and attach
// the launch's algorithmic byte count; query() resolves the pending events.
#pragma once

#include <hip/hip_runtime.h>

namespace ikr {

enum KernelId : int {
  K_COL_INV = 0,    // sphere -> column transforms (with fused p update)
  K_PLANE_HV = 1,   // plane 2D FFT pair with the local-potential multiply
  K_COL_FWD = 2,    // column forward transforms -> sphere, H epilogue
  K_GRAM = 3,       // projection coefficients W^H X
  K_UPDATE = 4,     // projection updates X + W C (with dot partials)
  K_CG_STEP = 5,    // fused CG vector update
  K_PLANE_RHO = 6,  // density accumulation
  K_FP32 = 7,       // FP32 variants of ids 0..5 follow: K_FP32 + id
  K_COUNT = 13
};

// Id of a CG kernel for the precision R (FP32 launches are timed apart).
template <typename R> constexpr int kid(int id) { return sizeof(R) == 4 ? K_FP32 + id : id; }

const char* kernel_name(int id);

struct KTimer {
  static void enable(unsigned kernel_mask);   // bit i times kernel i
  static bool enabled();
  static void begin(int id, hipStream_t st);
  static void end(int id, hipStream_t st, double bytes);
  // algorithmic bytes of launches whose size is known only after they ran
  static void add_bytes(int id, double bytes);
  // launches, total milliseconds and total algorithmic bytes since reset
  static void query(int id, long long* launches, double* ms, double* bytes);
  static void reset();
};

}  // namespace ikr
