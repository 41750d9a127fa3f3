// Internal interface between the C ABI (spme_api.cpp) and the kernels
// (spme_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace spme {

constexpr int kBinThreads = 1024;    // largest binning chunk (one atom per thread)
constexpr int kMinChunk = 256;       // smallest binning chunk
constexpr int kMaxBins = 2048;       // (z, y slice, head/body) bins: 2 K3 nq <= 2048
// threads of a spreading tile (one y slice of one z-plane per workgroup):
// 1024 for one system (halves each thread's chain of records), 512 for
// batched launches (where many tiles share each CU, measured faster)
constexpr int kSpreadThreads = 1024, kSpreadThreadsBatch = 512;
constexpr int kPlaneThreads = 512;   // one z-plane per workgroup (debug potential copy)
constexpr int kInterpThreads = 512;  // one (z-plane, y slice) bin per workgroup
constexpr int kMaxLds = 160 * 1024;  // LDS per workgroup on gfx950
constexpr int kNumKernels = 4;       // bin, spread+x, yz convolution, inverse x + interpolation

// y slices per z-plane for K2 points along y (rows per slice >= 8 > p - 1,
// so an atom's support reaches at most one slice below its own); FP64 at
// K2 = 128 uses narrower slices so that the interpolation tile fits in LDS.
__host__ __device__ constexpr int nq_of(int K2, bool fixed) {
  return (!fixed && K2 == 128) ? 8 : K2 >= 32 ? 4 : K2 / 8;
}
__host__ __device__ constexpr int phi_pitch_of(int K, int order) {
  return (K + order - 1 + 3) / 4 * 4;
}
// Records per bucket: twice the mean number of atoms per (z-plane, slice)
// of a grid with K3 planes, plus a margin; fuller buckets spill to the
// overflow list.
__host__ __device__ constexpr int bucket_cap(int K3, int nq, int max_atoms) {
  return (int)(((2 * (long long)max_atoms / (K3 * nq) + 64 + 31) / 32) * 32);
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
  size_t bsq;      // double[K1 + K2 + K3]: squared B-spline moduli per axis, x then y then z
  size_t tw;       // complex[K1 + K2 + K3]: exp(-2 pi i k/K_a) per axis, float2 or double2
  size_t bcnt;     // unsigned[2 K3 nq]: atoms binned so far per bucket (zero between steps)
  size_t bcnt2;    // unsigned[2 K3 nq]: this step's counts, kept for the interpolation
  size_t ovf;      // unsigned[4]: [0] overflow records so far, [1] this step's, kept
  size_t absq;     // double[n_chunks_max]: sum |q| per binning chunk (fixed-point headroom)
  size_t rec;      // records [2 K3 nq][cap] (RecF or RecD): one bucket per bin
  size_t orec;     // records [max_atoms]: atoms that found their bucket full
  size_t spec;     // complex[K1/2+1][K3][K2] half spectrum, columns [x'][z][y]
  size_t mid;      // complex[K1/2+1][K3][K2] at full precision between the split convolution
                   // passes of a binary16-spectrum plan; otherwise the same region as spec
  size_t phi;      // real[K3][K2][phi_pitch]: potential rows with a (p-1) wrap halo in front
  size_t partial;  // double[partial_rows][8]: energy/virial partial sums
  size_t dbg;      // int64 or double [K3][K2][K1]: charge-grid copy (debug)
  size_t args;     // Args: device copy of the bound step arguments (batched runs)
  size_t total;
  int n_chunks_max;
  int cap;          // records per bucket
  int orec_max;     // overflow records (max_atoms)
  int partial_rows;  // energy/virial rows: one per wavefront of the convolution (largest variant)
  int phi_pitch;
};

struct Args {
  int K1, K2, K3;  // grid points along x, y, z
  int order, precision, frac_bits;
  int N, n_chunks;
  int accumulate, keep_grid;
  int reduce_ev;  // the last launch's extra workgroup adds the energy/virial rows
  int conv_mode;    // kConvFused, kConvSplit or kConvReg
  int interp_mode;  // kInterpFused or kInterpSplit
  int bin_chunk;    // atoms per binning workgroup (kMinChunk .. kBinThreads, a multiple of 64)
  int ev_rows;      // energy/virial rows the convolution variant writes (from row 0)
  int triclinic;     // 0: diagonal box (L, invL); 1: general cell (rec)
  double L[3], invL[3];
  double rec[9];     // rec[3a + c]: component c of reciprocal vector a*_a
  double beta, coulomb, volume;
  const double* pos;
  const double* q;
  double* forces;
  double* ev;
  char* ws;
  Layout lay;
};

// Batched launches: device copies of the Args of up to kMaxBatch systems of
// one (precision, grid, order) group; workgroup (x, y) works on system y.
constexpr int kMaxBatch = 128;
struct BatchArgs {
  int n;
  const Args* sys[kMaxBatch];
};

// Variants of the y/z convolution and of the interpolation (a plan's
// tuning picks one of each among those its shape supports).
constexpr int kConvFused = 0;    // one workgroup per x' column, all y/z work in LDS
constexpr int kConvSplit = 1;    // three launches of row-chunk workgroups
constexpr int kConvReg = 2;      // one workgroup per column, transforms held in registers
constexpr int kInterpFused = 0;  // inverse x transform of a bin's rows + interpolation, one launch
constexpr int kInterpSplit = 1;  // inverse x transform per plane, then a gather launch
constexpr unsigned kVarConvFused = 1u, kVarConvSplit = 2u, kVarInterpFused = 4u,
                   kVarInterpSplit = 8u, kVarConvReg = 16u;

// Optional events attached to one kernel dispatch (both null: untimed).
struct Timing {
  hipEvent_t start = nullptr, stop = nullptr;
};

using LaunchFn = hipError_t (*)(const Args&, hipStream_t, const Timing&, const BatchArgs*);

// Launch table of one precision: its kernels are compiled in a translation
// unit of their own (spme_kern_<precision>.hip).
struct PrecOps {
  hipError_t (*prepare)(int K1, int K2, int K3, int order);  // dynamic-LDS limits
  unsigned (*variants)(int K1, int K2, int K3, int order);   // kVar* bits
  LaunchFn bin, spread_x, conv, inv_x, interp;
#ifdef SPME_TRACE
  hipError_t (*trace_set)(void* buf);
#endif
};
extern const PrecOps kOpsFixed, kOpsHalf, kOpsBf16, kOpsDouble;
const PrecOps* prec_ops(int precision);  // null for an unknown precision

bool grid_supported(int K1, int K2, int K3);
// Variants available to a plan (kVar* bits; 0 when unsupported), and the
// built-in choice of each.
unsigned variants_for(int K1, int K2, int K3, int order, int precision);
void default_variants(int K1, int K2, int K3, int order, int precision, int* conv_mode,
                      int* interp_mode);
bool layout_for(int K1, int K2, int K3, int order, int max_atoms, int precision, Layout* lay);
// Energy/virial rows a convolution variant writes (0 when unsupported).
int ev_rows_for(int K1, int K2, int K3, int precision, int conv_mode);

// Raise dynamic-LDS limits of the kernels a plan will launch.
hipError_t prepare_kernels(int K1, int K2, int K3, int order, int precision);

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
hipError_t launch_clear_counts(const Args& a, hipStream_t s);
hipError_t launch_clear_flags(const Args& a, hipStream_t s);

// Plan initialisation on the device: mp[k] = M_p(k + 1), k <= p - 2.
struct PlanInit {
  double mp[8];
};
hipError_t launch_init_plan(const Args& a, const PlanInit& in, hipStream_t s);
// Stream-ordered write of a system's arguments to their device copy.
hipError_t launch_store_args(const Args& a, Args* dst, hipStream_t s);

}  // namespace spme
