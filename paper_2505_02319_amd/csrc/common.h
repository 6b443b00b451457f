// Internal declarations shared by the HIP kernels and the host driver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

namespace ikr {

// ---------------------------------------------------------------- complex
template <typename R> struct cvec;
template <> struct cvec<double> { using type = double2; };
template <> struct cvec<float> { using type = float2; };
template <typename R> using cplx = typename cvec<R>::type;

template <typename R>
__host__ __device__ inline cplx<R> mk(R x, R y) { cplx<R> c; c.x = x; c.y = y; return c; }
template <typename R>
__host__ __device__ inline cplx<R> cadd(cplx<R> a, cplx<R> b) { return mk<R>(a.x + b.x, a.y + b.y); }
template <typename R>
__host__ __device__ inline cplx<R> csub(cplx<R> a, cplx<R> b) { return mk<R>(a.x - b.x, a.y - b.y); }
template <typename R>
__host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return mk<R>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <typename R>
__host__ __device__ inline cplx<R> cmulc(cplx<R> a, cplx<R> b) {
  return mk<R>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
template <typename R>
__host__ __device__ inline cplx<R> cscale(cplx<R> a, R s) { return mk<R>(a.x * s, a.y * s); }

// ---------------------------------------------------------------- errors
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define IKR_HIP(call)                                                          \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess)                                                      \
      throw ::ikr::Error(e_ == hipErrorOutOfMemory ? 6 : 7,                    \
                         std::string(#call) + ": " + hipGetErrorString(e_));  \
  } while (0)

#define IKR_CHECK(cond, code, msg)                                             \
  do {                                                                         \
    if (!(cond)) throw ::ikr::Error((code), (msg));                           \
  } while (0)

// ---------------------------------------------------------------- geometry
// Device view of the plane-wave spheres and the internal grid layout.
// The internal real-space layout is [C][P][Q] (Q fastest): C is the column
// axis of the pruned transform, (P, Q) the in-LDS plane.  Column buffers
// ("T buffers") are [C][ncol_max] per vector: for each c, the footprint
// columns of the sphere on the (P, Q) plane.
struct Geom {
  int C, P, Q;
  int nk;
  int nb_max;
  int ncol_max;
  const int* nb;         // [nk]
  const int* ncol;       // [nk]
  const int* col_start;  // [nk][ncol_max + 1] offsets into the basis order
  const int* col_pq;     // [nk][ncol_max] plane index p*Q + q of the column
  const int* col_clo;    // [nk][ncol_max] first (signed) c index of the column
  const double* kin;     // [nk][nb_max] |G+k|^2/2, 0 beyond nb
  const int* prow = nullptr;   // [nk][P] rows p of the plane that hold columns, ascending
  const int* nprow = nullptr;  // [nk] their number
};

// Per-slot (band of the batch) metadata for batched kernels.  A launch
// covers n grid rows; row y works on slot list[y] (list may be null: y).
struct Slots {
  int n;                 // number of grid rows (an upper bound when dn is set)
  const int* k;          // [slots] k-point of the slot
  const int* active;     // [slots] nonzero when the slot takes part (may be null)
  const int* list = nullptr;   // [n] compact list of slots (may be null)
  const int* dn = nullptr;     // device count of live rows (may be null: all n)
};

// Work item of block `b` of a 1D launch of `nblk` blocks (a multiple of 8):
// blocks are dealt round-robin to the 8 XCDs, so XCD x is given the
// contiguous items [x * nblk / 8, (x + 1) * nblk / 8).  Items that share
// operands are numbered consecutively by the caller and so run back to back
// on one XCD, where they meet in its L2.
__device__ __forceinline__ int xcd_item(int b, int nblk) {
  return (b & 7) * (nblk >> 3) + (b >> 3);
}
inline int round8(int n) { return (n + 7) / 8 * 8; }

__device__ __forceinline__ int slot_of(const Slots& s, int row) {
  return s.list ? s.list[row] : row;
}

// False for grid rows past the device-side live count.
__device__ __forceinline__ bool row_live(const Slots& s, int row) {
  return !s.dn || row < *s.dn;
}

// ---------------------------------------------------------------- FFT API
// All transforms are unnormalised: inverse = sum_G x_G e^{+iG.r},
// forward = sum_r x_r e^{-iG.r}.
bool fft_length_supported(int n);

// Twiddle tables live in one device buffer built at setup.
struct FftTables {
  double2* tw64 = nullptr;   // concatenated tables e^{-2 pi i m / N}
  float2* tw32 = nullptr;
  int offC = 0, offP = 0, offQ = 0;
};

enum PlaneMode : int {
  PLANE_HV = 0,   // T -> inverse 2D -> * V (real) -> forward 2D -> T
  PLANE_FWD = 1,  // real grid -> forward 2D -> T (full footprint)
  PLANE_INV = 2,  // T (full) -> inverse 2D -> real part -> grid (+ epilogue)
  PLANE_RHO = 3,  // T_a, T_b -> inverse 2D both -> accumulate density terms
  PLANE_GRID = 4  // T -> inverse 2D -> complex grid out
};

template <typename R>
void launch_col_inv(const Geom& g, const FftTables& t, const Slots& s,
                    const cplx<R>* x, int x_stride, cplx<R>* T,
                    const cplx<R>* z, const R* beta, cplx<R>* pout,
                    hipStream_t st);

template <typename R>
void launch_col_fwd(const Geom& g, const FftTables& t, const Slots& s,
                    const cplx<R>* T, cplx<R>* y, int y_stride,
                    const cplx<R>* x, const R* shift, R scale, hipStream_t st);

// pt: threads per plane block (0: by shape; 256 or 512 where both are built,
// the planes of 48 x 48 points and larger)
template <typename R>
void launch_plane_hv(const Geom& g, const FftTables& t, const Slots& s,
                     const cplx<R>* Tin, cplx<R>* Tout, const R* V,
                     int v_per_slot, hipStream_t st, int pt = 0);
// Threads per plane block that launch_plane_hv takes for pt on this plane.
int plane_hv_threads(const Geom& g, int pt, bool fp64);

// Density accumulation: for slots in [s0, s0+ns), with weights wa[slot]
// (2 f w_k / |Omega|) and wb[slot] (delta f w_k / |Omega|):
//   part[grp][r] = sum_{slots of group} wa Re(conj(a) b) + wb |a|^2,
// a = inverse 2D of Ta, b = inverse 2D of Tb; groups of gsize slots.
void launch_plane_rho(const Geom& g, const FftTables& t, int nslots,
                      const int* slot_k, const double2* Ta, const double2* Tb,
                      const double* wa, const double* wb, int gsize,
                      double* part, hipStream_t st);

// Complex grid of each slot (inverse of the T buffer), layout [C][P][Q].
void launch_plane_grid(const Geom& g, const FftTables& t, int nslots,
                       const int* slot_k, const double2* T, double2* grid,
                       hipStream_t st);

// Full-grid real transform pipeline used by the Hxc kernel:
// out = Re IFFT(khat * FFT(v)) / N_g + fx * v, and per-plane partial
// sums of out^2 (for ||K v||).  v, out in the internal layout.
void launch_kernel_apply(const Geom& g, const FftTables& t, const double* v,
                         const double* khat, const double* fx, double* out,
                         double2* work1, double2* work2, double* partial,
                         hipStream_t st);

}  // namespace ikr
