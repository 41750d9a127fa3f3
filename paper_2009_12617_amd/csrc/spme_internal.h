// Internal interface between the C ABI (spme_api.cpp) and the kernels
// (spme_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace spme {

constexpr int kChunk = 1024;         // atoms per binning workgroup (one sorted chunk)
constexpr int kBinThreads = 1024;    // one atom per thread
constexpr int kMaxBins = 1024;       // (z, y slice, head/body) bins per chunk: 2 K nq <= 1024
constexpr int kItemMap = 4096;       // items per window of the spreading item map
constexpr int kSegPerThread = 4;     // spreading segments described per thread per batch
constexpr int kSpreadThreads = 512;  // one y slice of one z-plane per workgroup
constexpr int kPlaneThreads = 512;   // one z-plane per workgroup
constexpr int kInterpThreads = 512;  // one (z-plane, y slice) bin per workgroup
constexpr int kInterpItems = 2048;   // atoms per window of the interpolation item list
constexpr int kGatherThreads = 256;  // one atom per thread
constexpr int kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kNumKernels = 5;       // bin, spread+x, yz convolution, inverse x, interpolation

// y slices per z-plane in the spreading pass (rows per slice >= 8 > p - 1,
// so an atom's support reaches at most one slice below its own).
__host__ __device__ constexpr int nq_of(int K) { return K >= 32 ? 4 : K / 8; }
__host__ __device__ constexpr int phi_pitch_of(int K, int order) {
  return (K + order - 1 + 3) / 4 * 4;
}

// Sorted atom record of the FP32/fixed path (32 bytes): packed base grid
// index (x | y << 10 | z << 20), single-precision fractional offsets and
// charge (spreading), index of the atom in the caller's order, and the
// double-precision charge (interpolation).
struct RecF {
  int g;
  float w[3];
  float q;
  int idx;
  double qd;
};
// FP64 path (48 bytes).
struct RecD {
  int g;
  int idx;
  double w[3];
  double q;
  double qd;  // same as q
};

// Byte offsets of the workspace regions (each 256-byte aligned).
struct Layout {
  size_t ctrl;     // unsigned[64]: [0] sticky flags
  size_t bsq;      // double[3][K]: squared B-spline moduli per axis
  size_t tw;       // complex[K]: exp(-2 pi i k/K), float2 or double2
  size_t cnt;      // int2[n_chunks][2 K nq]: (count, offset within the chunk) of the
                   // atoms of chunk c in bin (z, y slice, head/body)
  size_t absq;     // double[n_chunks]: sum |q| per chunk (fixed-point headroom)
  size_t rec;      // records [n_chunks * kChunk] (RecF or RecD)
  size_t spec;     // complex[K/2+1][K][K] half spectrum, columns [x'][z][y]
  size_t phi;      // real[K][K][phi_pitch]: potential rows with a (p-1) wrap halo in front
  size_t partial;  // double[conv_blocks][8]: energy/virial partial sums
  size_t dbg;      // int64 or double [K][K][K]: charge-grid copy (debug)
  size_t args;     // Args: device copy of the bound step arguments (batched runs)
  size_t total;
  int n_chunks_max;
  int conv_blocks;  // K/2+1 columns, one partial row each
  int phi_pitch;
};

struct Args {
  int K, order, precision, frac_bits;
  int N, n_chunks;
  int accumulate, keep_grid;
  int reduce_ev;  // the last launch's extra workgroup adds the energy/virial rows
  double L[3], invL[3];
  double beta, coulomb, volume;
  const double* pos;
  const double* q;
  double* forces;
  double* ev;
  char* ws;
  Layout lay;
};

// Batched launches: device copies of the Args of up to kMaxBatch systems of
// one (precision, K, order) group; workgroup (x, y) works on system y.
constexpr int kMaxBatch = 128;
struct BatchArgs {
  int n;
  const Args* sys[kMaxBatch];
};

// Optional events attached to one kernel dispatch (both null: untimed).
struct Timing {
  hipEvent_t start = nullptr, stop = nullptr;
};

bool grid_supported(int K);
bool layout_for(int K, int order, int max_atoms, int precision, Layout* lay);

// Raise dynamic-LDS limits of the kernels a plan will launch.
hipError_t prepare_kernels(int K, int order, int precision);

hipError_t launch_bin(const Args& a, hipStream_t s, const Timing& t = Timing(),
                      const BatchArgs* bt = nullptr);
hipError_t launch_spread_x(const Args& a, hipStream_t s, const Timing& t = Timing(),
                      const BatchArgs* bt = nullptr);
hipError_t launch_conv(const Args& a, hipStream_t s, const Timing& t = Timing(),
                       const BatchArgs* bt = nullptr);
hipError_t launch_reduce_ev(const Args& a, hipStream_t s);
hipError_t launch_inv_x(const Args& a, hipStream_t s, const Timing& t = Timing(),
                        const BatchArgs* bt = nullptr);
hipError_t launch_interp(const Args& a, hipStream_t s, const Timing& t = Timing(),
                         const BatchArgs* bt = nullptr);
hipError_t launch_gather(const Args& a, hipStream_t s, const Timing& t = Timing(),
                         const BatchArgs* bt = nullptr);
// Whether the inverse x transform and interpolation run as one launch
// (k_interp) for these parameters, or as k_inv_x + k_gather.
bool interp_is_fused(int K, int order, int precision);
hipError_t launch_clear_flags(const Args& a, hipStream_t s);

}  // namespace spme
