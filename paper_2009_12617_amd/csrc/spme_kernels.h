// HIP kernels of the SPME reciprocal-space step for gfx950 (CDNA4).
//
// One step is four launches on one stream (more on large grids, below):
//   k_bin       fractional coordinates, base grid index and offsets of each
//               atom; the atoms are put into buckets by (base z, y slice,
//               head/body) -- the GPU counterpart of the paper's atom
//               reordering for hazard suppression (§III.A.1, §V.C)
//   k_spread_x  one y slice of one z-plane per workgroup: every atom whose
//               support covers the slice adds its contributions into an LDS
//               tile in 64-bit fixed point (integer adds commute, so the grid
//               is bit-identical whatever the order); the finished rows are
//               converted to FP32, transformed along x (real-to-complex) and
//               stored as columns [x'][z][y] of the half spectrum
//   k_conv      one x' column per workgroup: y and z transforms, the
//               influence function with FP64 energy and virial partials,
//               inverse z and y transforms (§III.A.2); one extra workgroup
//               keeps the bucket counts for k_interp and clears them
//   k_interp    one (z-plane, y-slice) bin per workgroup: complex-to-real x
//               transforms of the p planes and p-1+R rows that the bin's
//               atoms touch, then force interpolation from LDS, forces
//               scattered back to the caller's atom order (§III.A.3); one
//               extra workgroup adds the energy/virial partial rows
// The paper's two all-to-all corner turns (§III.A.2, §IV.C) become the
// column layout of the half spectrum: each column holds every y and z of one
// x', so both turns happen inside k_conv.  Two variants replace a launch by
// several where that pays (a plan picks them, by default or by measurement):
// the column work split over three launches (k_conv_y, k_conv_z, k_conv_y;
// the default for K2 K3 >= 8192), and the inverse x transform run once per
// plane (k_inv_x, which also serves the debug copy of the potential) before
// a gather kernel (k_interp_phi; the default for p >= 6 on K2 K3 >= 16384).
#pragma once

#include <hip/hip_ext.h>

#include <type_traits>

#include "spme_device.h"
#include "spme_internal.h"
#include "../../include/spme.h"

namespace spme {

// Optional phase trace (build with -DSPME_TRACE): thread 0 of each workgroup
// stamps the 100 MHz wall clock at phase boundaries into
// trace[kernel][workgroup][phase]; kernels 0..4 as in the timing order, phase 0 at
// entry and 15 at exit.
#ifdef SPME_TRACE
static __device__ unsigned long long* g_trace;
// points this translation unit's trace at a device buffer (or NULL)
static inline hipError_t trace_set_here(void* buf) {
  unsigned long long* p = static_cast<unsigned long long*>(buf);
  return hipMemcpyToSymbol(HIP_SYMBOL(g_trace), &p, sizeof(p));
}
#define TRACE(kernel, phase)                                                         \
  do {                                                                               \
    if (threadIdx.x == 0 && g_trace != nullptr && blockIdx.x < 1024)                 \
      g_trace[((size_t)(kernel) * 1024 + blockIdx.x) * 16 + (phase)] = wall_clock64(); \
  } while (0)
#else
#define TRACE(kernel, phase) \
  do {                       \
  } while (0)
#endif

// Half-spectrum storage between launches: complex float, complex double, or
// (reduced-precision variants) a pair of IEEE binary16 values, or a pair of
// bfloat16 values (the upper 16 bits of an FP32), rounded to nearest even.
struct cplx_h {
  _Float16 x, y;
};
struct cplx_b {
  unsigned short x, y;
};
// FP32 -> bfloat16, round to nearest, ties to even: add 0x7fff plus the
// kept part's lowest bit, then truncate.  Finite inputs only (the spectrum
// of a finite grid); values within half a bfloat16 step of FLT_MAX round to
// infinity as the rule says.
__device__ __forceinline__ unsigned short bf16_rne(float v) {
  const unsigned u = __float_as_uint(v);
  return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_up(unsigned short h) {
  return __uint_as_float((unsigned)h << 16);
}
__device__ __forceinline__ cplx<float> spec_ld(const cplx<float>* p) { return *p; }
__device__ __forceinline__ cplx<double> spec_ld(const cplx<double>* p) { return *p; }
__device__ __forceinline__ cplx<float> spec_ld(const cplx_h* p) {
  const cplx_h h = *p;
  return {(float)h.x, (float)h.y};
}
__device__ __forceinline__ void spec_st(cplx<float>* p, cplx<float> v) { *p = v; }
__device__ __forceinline__ void spec_st(cplx<double>* p, cplx<double> v) { *p = v; }
__device__ __forceinline__ void spec_st(cplx_h* p, cplx<float> v) {
  *p = cplx_h{(_Float16)v.x, (_Float16)v.y};
}
__device__ __forceinline__ cplx<float> spec_ld(const cplx_b* p) {
  const cplx_b h = *p;
  return {bf16_up(h.x), bf16_up(h.y)};
}
__device__ __forceinline__ void spec_st(cplx_b* p, cplx<float> v) {
  *p = cplx_b{bf16_rne(v.x), bf16_rne(v.y)};
}

struct PFixed {
  using real = float;
  using acc = unsigned long long;
  using rec = RecF;
  using spec = cplx<float>;
  static constexpr bool fixed = true;
};
// FP32/fixed with the half spectrum kept in FP16 between launches
struct PHalf {
  using real = float;
  using acc = unsigned long long;
  using rec = RecF;
  using spec = cplx_h;
  static constexpr bool fixed = true;
};
// FP32/fixed with the half spectrum kept in bfloat16 between launches
struct PBf16 {
  using real = float;
  using acc = unsigned long long;
  using rec = RecF;
  using spec = cplx_b;
  static constexpr bool fixed = true;
};
struct PDouble {
  using real = double;
  using acc = double;
  using rec = RecD;
  using spec = cplx<double>;
  static constexpr bool fixed = false;
};

// Grid shape as a type: K1, K2, K3 points along x, y, z.
template <int A, int B, int C>
struct Grid {
  static constexpr int K1 = A, K2 = B, K3 = C;
};

// Row pitch of an LDS grid tile (one x row of K points) in 8-byte units.
// Fixed point: at least K int64 values per row (the half spectrum of K/2+1
// float2 fits in place).
// FP64: room for K/2+1 double2.  The padding skews rows across LDS banks.
template <class P>
__host__ __device__ constexpr int tile_pitch(int K) {
  // chosen with a bank model of the x transform's Stockham stages over rows
  // of this pitch (64-lane wavefront, 4-byte banks)
  return P::fixed ? (K == 32 ? 34 : K == 64 ? 66 : K == 96 ? 98 : K == 128 ? 135 : K + 1)
                  : 2 * (K == 128 ? 71 : K / 2 + 1);
}

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap workgroup b of n (n a multiple of 8) so that XCD b % 8 owns the
// contiguous block of logical indices [(b % 8) n/8, (b % 8 + 1) n/8): z-planes
// that share atoms then share one L2.
constexpr int kXcds = 8;
__device__ __forceinline__ int xcd_local(int b, int n) {
  return (b % kXcds) * (n / kXcds) + b / kXcds;
}

template <int P, typename T>
__device__ __forceinline__ T pick(const T* a, int i) {
  // a[i] for a register array and a lane-varying i, written as a masked sum
  // (a[i] plus exact zeros) so that the array stays in registers
  T v = T(0);
#pragma unroll
  for (int k = 0; k < P; ++k) v += a[k] * T(i == k ? 1 : 0);
  return v;
}

// ---------------------------------------------------------------------------
// k_bin: one chunk of atoms per workgroup (the plan's binning chunk, 256 to
// 1024 atoms), one atom per thread.  Each
// atom goes to the bucket of its bin (base z, y slice, head/body); a bucket
// is a fixed run of `cap` records.  The chunk counts its atoms per bin in
// LDS, reserves that many slots of each bucket with one global add, and
// writes its records there; atoms beyond a full bucket go to the overflow
// list, which every consumer also scans.  The order of records inside a
// bucket varies from run to run; nothing downstream depends on it (the grid
// is an order-free integer sum, forces are per atom).
// ---------------------------------------------------------------------------
template <class P, bool BATCH>
__global__ __launch_bounds__(kBinThreads) void k_bin(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  if (BATCH && (int)blockIdx.x >= a.n_chunks) return;
  using Rec = typename P::rec;
  using T = typename P::real;
  __shared__ int hist[kMaxBins];
  __shared__ double wred[16 * 8];
  TRACE(0, 0);
  const int nq = nq_of(a.K2, P::fixed), rows = a.K2 / nq, nbins = 2 * a.K3 * nq;
  const int cap = a.lay.cap;
  const int c = blockIdx.x, tid = threadIdx.x;
  unsigned* bcnt = reinterpret_cast<unsigned*>(a.ws + a.lay.bcnt);
  unsigned* ovf = reinterpret_cast<unsigned*>(a.ws + a.lay.ovf);
  Rec* rec = reinterpret_cast<Rec*>(a.ws + a.lay.rec);
  Rec* orec = reinterpret_cast<Rec*>(a.ws + a.lay.orec);
  unsigned* flags = reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl);
  const int nt = blockDim.x;  // atoms per chunk
  for (int b = tid; b < nbins; b += nt) hist[b] = 0;
  __syncthreads();
  TRACE(0, 1);

  const int i = c * nt + tid;
  Rec r;
  int bin = -1, rank = 0;
  double v[1] = {0.0};
  if (i < a.N) {
    int g[3];
    double w[3];
    bool ok = true;
    const double x3[3] = {a.pos[3 * (size_t)i], a.pos[3 * (size_t)i + 1], a.pos[3 * (size_t)i + 2]};
    if (!a.triclinic) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int Kd = d == 0 ? a.K1 : d == 1 ? a.K2 : a.K3;
        ok &= grid_coord(x3[d], a.invL[d], Kd, &g[d], &w[d]);
      }
    } else {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        const int Kd = d == 0 ? a.K1 : d == 1 ? a.K2 : a.K3;
        ok &= grid_coord_s(frac_general(x3, a.rec + 3 * d), Kd, &g[d], &w[d]);
      }
    }
    double qi = a.q[i];
    ok &= (qi - qi == 0.0);  // finite
    if (!ok) {
      qi = 0.0;  // contributes nothing; reported through the sticky flag
      atomicOr(flags, PME_FLAG_NONFINITE);
    }
    v[0] = fabs(qi);
    r.g = g[0] | (g[1] << 10) | (g[2] << 20);
    r.w[0] = (T)w[0];
    r.w[1] = (T)w[1];
    r.w[2] = (T)w[2];
    r.q = (T)qi;
    r.qd = qi;
    r.idx = i;
    // bin (z, y slice, head/body): the head holds the atoms whose support
    // also reaches the slice below (g_y mod rows < p - 1)
    const int sl = g[1] / rows;
    bin = (g[2] * nq + sl) * 2 + ((g[1] - sl * rows) >= a.order - 1 ? 1 : 0);
    rank = atomicAdd(&hist[bin], 1);
  }
  // sum |q| of the chunk (fixed-point headroom); its barrier also completes
  // the histogram
  block_sums<1>(v, wred);
  TRACE(0, 2);
  for (int b = tid; b < nbins; b += nt) {
    const int h = hist[b];
    if (h > 0) hist[b] = (int)atomicAdd(&bcnt[b], (unsigned)h);
  }
  __syncthreads();
  TRACE(0, 3);
  if (bin >= 0) {
    const int slot = hist[bin] + rank;
    if (slot < cap) {
      rec[(size_t)bin * cap + slot] = r;
    } else {
      const unsigned o = atomicAdd(&ovf[0], 1u);
      if (o < (unsigned)a.lay.orec_max)
        orec[o] = r;
      else  // counts left over from a step that never reached its convolution
        atomicOr(flags, PME_FLAG_BUCKETS);
    }
  }
  if (tid == 15) reinterpret_cast<double*>(a.ws + a.lay.absq)[c] = v[0];
  TRACE(0, 15);
}

// The twiddles lane j (< R) of a register-resident N-point transform
// (N = 8 R) uses, kept in registers: wf[s] = W^(j s), s < 8, for the forward
// direction and wi[eR + l] = W^(l (jE + e)), l < R, e < E = 8/R, for the
// inverse one, W = exp(-2 pi i / N) from the table tw[k] = W^k (for R = 8 the
// two sets coincide).
template <typename T, int N>
struct RegTw {
  static constexpr int R = N / 8, E = 8 / R;
  cplx<T> wf[8], wi[8];
  // STEP: table stride (a table of W_{STEP N}^k serves the N-point transform)
  template <int STEP = 1>
  __device__ __forceinline__ void load(int j, const cplx<T>* tw) {
#pragma unroll
    for (int s = 1; s < 8; ++s) wf[s] = tw[STEP * j * s];
    if constexpr (R == 8) {
#pragma unroll
      for (int l = 1; l < 8; ++l) wi[l] = wf[l];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e)
#pragma unroll
        for (int l = 1; l < R; ++l) wi[e * R + l] = tw[STEP * l * (j * E + e)];
    }
  }
};

// Forward (S = -1) or inverse (S = +1) N-point DFT, N = 8 R, of the pencil
// whose points j + R r (r < 8) lane j (< R) holds in v[r]; on return v[eR + t]
// holds mode jE + e + 8t.  scr: the pencil's LDS scratch (R rows of pitch
// 9, starting at the pencil's first lane x 9); w: the lane's twiddles.
template <typename T, int N, int S>
__device__ __forceinline__ void rfft_fwd(cplx<T>* v, int j, cplx<T>* scr, const RegTw<T, N>& w) {
  constexpr int R = N / 8, E = 8 / R;
  Dft<8, S, T>::run(v);
#pragma unroll
  for (int s = 1; s < 8; ++s) v[s] = S < 0 ? c_mul(v[s], w.wf[s]) : c_mulc(v[s], w.wf[s]);
#pragma unroll
  for (int s = 0; s < 8; ++s) scr[j * 9 + s] = v[s];
  lds_order();
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int l = 0; l < R; ++l) v[e * R + l] = scr[l * 9 + j * E + e];
  lds_order();
#pragma unroll
  for (int e = 0; e < E; ++e) Dft<R, S, T>::run(v + e * R);
}

// The inverse direction of rfft_fwd's layouts: v[eR + t] holds mode
// jE + e + 8t on entry; on return v[r] holds point j + R r.
template <typename T, int N, int S>
__device__ __forceinline__ void rfft_inv(cplx<T>* v, int j, cplx<T>* scr, const RegTw<T, N>& w) {
  constexpr int R = N / 8, E = 8 / R;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    Dft<R, S, T>::run(v + e * R);
#pragma unroll
    for (int l = 1; l < R; ++l)
      v[e * R + l] = S < 0 ? c_mul(v[e * R + l], w.wi[e * R + l]) : c_mulc(v[e * R + l], w.wi[e * R + l]);
  }
#pragma unroll
  for (int e = 0; e < E; ++e)
#pragma unroll
    for (int l = 0; l < R; ++l) scr[l * 9 + j * E + e] = v[e * R + l];
  lds_order();
#pragma unroll
  for (int s = 0; s < 8; ++s) v[s] = scr[j * 9 + s];
  lds_order();
  Dft<8, S, T>::run(v);
}


// Register-resident x transforms of one row of K1 = 2M reals (M = 32 or 64):
// the M-point complex transform of the packed sequence z_n = x_{2n} +
// i x_{2n+1} runs in registers (rfft_fwd / rfft_inv, RX = M/8 lanes per row,
// lane j holding points j + RX r), the packing identities of r2c_post and
// c2r_pre go through the row in LDS.  The decomposition (radix 8, twiddles
// W_M^(j s), radix RX) and the twiddle table entries are those of the
// Stockham stages of fft_pencil for these lengths.
template <int K1>
__host__ __device__ constexpr bool reg_x_ok() {
  return K1 == 64 || K1 == 128;
}

// Forward: v holds points j + RX r of the row; the half spectrum X_0 .. X_M
// goes to sink(k, X_k) (each k once, over the row's lanes); the row (complex,
// in LDS) is overwritten with the M-point transform on the way.  scr: the
// row's scratch (RX rows of pitch 9); tw: W_K1^k, k < K1.  Every lane of the
// row must be in one wavefront.
template <typename T, int K1, class Sink>
__device__ __forceinline__ void r2c_row_reg(cplx<T>* v, cplx<T>* row, int j, cplx<T>* scr,
                                            const cplx<T>* tw, Sink&& sink) {
  constexpr int M = K1 / 2, RX = M / 8, EX = 8 / RX;
  RegTw<T, M> w;
  w.template load<2>(j, tw);
  rfft_fwd<T, M, -1>(v, j, scr, w);
  lds_order();
#pragma unroll
  for (int e = 0; e < EX; ++e)
#pragma unroll
    for (int t = 0; t < RX; ++t) row[j * EX + e + 8 * t] = v[e * RX + t];
  lds_order();
  r2c_post<T, K1>(row, j, tw, sink);
}

// Inverse: the row (complex, in LDS) holds X_0 .. X_M of a real row; on
// return it holds z_n = x_{2n} + i x_{2n+1}, n < M (unnormalised).  The
// c2r_pre identity is formed per mode in registers (Im X_0, Im X_M dropped).
template <typename T, int K1>
__device__ __forceinline__ void c2r_row_reg(cplx<T>* row, int j, cplx<T>* scr, const cplx<T>* tw) {
  constexpr int M = K1 / 2, RX = M / 8, EX = 8 / RX;
  cplx<T> v[8];
#pragma unroll
  for (int e = 0; e < EX; ++e)
#pragma unroll
    for (int t = 0; t < RX; ++t) {
      const int k = j * EX + e + 8 * t;
      cplx<T> xk = row[k], xm = row[M - k];
      if (k == 0) {
        xk.y = T(0);
        xm.y = T(0);
      }
      const cplx<T> am = c_add(xk, c_conj(xm));
      const cplx<T> bm = c_mulc(c_sub(xk, c_conj(xm)), tw[k]);
      v[e * RX + t] = {am.x - bm.y, am.y + bm.x};  // A + i B
    }
  RegTw<T, M> w;
  w.template load<2>(j, tw);
  lds_order();
  rfft_inv<T, M, 1>(v, j, scr, w);
#pragma unroll
  for (int r = 0; r < 8; ++r) row[j + RX * r] = v[r];
  lds_order();
}

// ---------------------------------------------------------------------------
// k_spread_x: charge spreading of one y slice of one z-plane, then the x
// real-to-complex FFT of its rows.
// ---------------------------------------------------------------------------
template <class P, class G>
__host__ __device__ constexpr size_t spread_lds_bytes() {
  // the tile, the twiddles, the bucket table, then (register x transforms)
  // the rows' transpose scratch: 9 complex per lane
  constexpr size_t R = G::K2 / nq_of(G::K2, P::fixed);
  return R * tile_pitch<P>(G::K1) * 8 + (size_t)G::K1 * sizeof(cplx<typename P::real>) +
         64 * sizeof(int) +
         (reg_x_ok<G::K1>() ? R * (G::K1 / 16) * 9 * sizeof(cplx<typename P::real>) : 0);
}

// Contributions of one atom to the plane of support point jz (z order) of
// the tile holding rows y0 .. y0+R-1: its p x p (y, x) points in the slice,
// in the product order z, y, x; fixed point: rounded to integers and added
// with 64-bit LDS atomics.
template <class P, int K1, int K2, int ORDER, int R, int PITCH>
__device__ __forceinline__ void spread_atom(typename P::acc* tile, const typename P::rec& r, int jz,
                                            int y0, double scale) {
  using T = typename P::real;
  using Acc = typename P::acc;
  const int gx = r.g & 1023, gy = (r.g >> 10) & 1023;
  T tx[ORDER], ty[ORDER], tz[ORDER];
  bspline<ORDER>(r.w[0], tx, (T*)nullptr);
  bspline<ORDER>(r.w[1], ty, (T*)nullptr);
  bspline<ORDER>(r.w[2], tz, (T*)nullptr);
  int xs[ORDER];
#pragma unroll
  for (int jx = 0; jx < ORDER; ++jx) {
    const int x = gx - ORDER + 1 + jx;
    xs[jx] = x < 0 ? x + K1 : x;
  }
  if constexpr (P::fixed) {
#pragma clang fp contract(off)
    const float cz = r.q * pick<ORDER>(tz, jz);
#pragma unroll
    for (int jy = 0; jy < ORDER; ++jy) {
      int dy = gy - ORDER + 1 + jy - y0;
      if (dy < 0) dy += K2;
      if (dy >= R) continue;
      Acc* row = tile + dy * PITCH;
      const float cy = cz * ty[jy];
#pragma unroll
      for (int jx = 0; jx < ORDER; ++jx)
        atomicAdd(&row[xs[jx]], (unsigned long long)to_fixed(cy * tx[jx], scale));
    }
  } else {
    const double cz = r.q * pick<ORDER>(tz, jz);
#pragma unroll
    for (int jy = 0; jy < ORDER; ++jy) {
      int dy = gy - ORDER + 1 + jy - y0;
      if (dy < 0) dy += K2;
      if (dy >= R) continue;
      Acc* row = tile + dy * PITCH;
      const double cy = cz * ty[jy];
#pragma unroll
      for (int jx = 0; jx < ORDER; ++jx) atomicAdd(&row[xs[jx]], cy * tx[jx]);
    }
  }
}

template <bool BATCH>
__host__ __device__ constexpr int spread_threads() {
  return BATCH ? kSpreadThreadsBatch : kSpreadThreads;
}

template <class P, class G, int ORDER, bool BATCH>
__global__ __launch_bounds__(spread_threads<BATCH>()) void k_spread_x(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  constexpr int NTS = spread_threads<BATCH>();
  using T = typename P::real;
  using Acc = typename P::acc;
  using Rec = typename P::rec;
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  constexpr int M = K1 / 2, KH = K1 / 2 + 1;
  constexpr int NQ = nq_of(K2, P::fixed), R = K2 / NQ;
  constexpr int PITCH = tile_pitch<P>(K1);
  constexpr int NBK = 3 * ORDER;  // buckets read per tile
  extern __shared__ __align__(16) unsigned char smem[];
  Acc* tile = reinterpret_cast<Acc*>(smem);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + (size_t)R * PITCH * 8);
  int* bk_pre = reinterpret_cast<int*>(tw + K1);  // [NBK + 1] item offsets
  int* bk_base = bk_pre + 24;                     // [NBK] first record
  int* bk_n = bk_base + 20;                       // [NBK] counts, then the overflow count
  cplx<T>* xscr = reinterpret_cast<cplx<T>*>(bk_pre + 64);  // register x transforms

  TRACE(1, 0);
  static_assert((K3 * NQ) % kXcds == 0, "spreading tiles do not split over the XCDs");
  const int tile_id = xcd_local(blockIdx.x, K3 * NQ);
  const int z = tile_id / NQ, qs = tile_id - z * NQ, y0 = qs * R;
  const int tid = threadIdx.x;
  const int cap = a.lay.cap;
  const unsigned* bcnt = reinterpret_cast<const unsigned*>(a.ws + a.lay.bcnt);
  const Rec* rec = reinterpret_cast<const Rec*>(a.ws + a.lay.rec);
  const Rec* orec = reinterpret_cast<const Rec*>(a.ws + a.lay.orec);
  // The tile (rows y0 .. y0+R-1 of plane z) receives the atoms whose base z
  // index b lies in z .. z+p-1 (mod K3) -- for b = z + j the plane is support
  // point jz = p-1-j -- and whose base y index lies in this slice, or in the
  // head (first p-1 rows) of the next slice: an atom touches rows
  // g_y-p+1 .. g_y.  Bucket k = 3j + d: d = 0 own head, 1 own body, 2 next
  // slice's head.
  if (tid < NBK) {
    const int j = tid / 3, d = tid - 3 * j;
    int bz = z + j;
    if (bz >= K3) bz -= K3;
    int by = qs + (d == 2 ? 1 : 0);
    if (by >= NQ) by -= NQ;
    const int b = (bz * NQ + by) * 2 + (d == 1 ? 1 : 0);
    bk_n[tid] = min((int)bcnt[b], cap);
    bk_base[tid] = b * cap;
  } else if (tid == NBK) {
    bk_n[NBK] = (int)min(reinterpret_cast<const unsigned*>(a.ws + a.lay.ovf)[0],
                         (unsigned)a.lay.orec_max);
  }
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < K1; i += NTS) tw[i] = twg[i];
  for (int i = tid; i < R * PITCH; i += NTS) tile[i] = Acc(0);
  const double scale = ldexp(1.0, a.frac_bits);
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int k = 0; k < NBK; ++k) {
      bk_pre[k] = run;
      run += bk_n[k];
    }
    bk_pre[NBK] = run;
  }
  __syncthreads();
  TRACE(1, 1);

  // items: the records of the buckets one after another; kItems per thread
  // per pass so that their loads overlap
  constexpr int kItems = 4;
  const int total = bk_pre[NBK];
  int pre[NBK + 1];
#pragma unroll
  for (int k = 0; k <= NBK; ++k) pre[k] = bk_pre[k];
  for (int it = 0; it < total; it += kItems * NTS) {
    int idx[kItems], jz[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u) {
      const int t = it + u * NTS + tid;
      jz[u] = -1;
      idx[u] = 0;
      if (t < total) {
        int k = 0;
#pragma unroll
        for (int kk = 1; kk < NBK; ++kk) k += (t >= pre[kk]) ? 1 : 0;
        idx[u] = bk_base[k] + (t - bk_pre[k]);
        jz[u] = ORDER - 1 - k / 3;
      }
    }
    Rec r[kItems];
#pragma unroll
    for (int u = 0; u < kItems; ++u)
      if (jz[u] >= 0) r[u] = rec[idx[u]];
#pragma unroll
    for (int u = 0; u < kItems; ++u)
      if (jz[u] >= 0) spread_atom<P, K1, K2, ORDER, R, PITCH>(tile, r[u], jz[u], y0, scale);
  }
  // atoms of full buckets: the whole overflow list, each atom taken if it
  // belongs to this tile
  const int novf = bk_n[NBK];
  for (int o = tid; o < novf; o += NTS) {
    const Rec r = orec[o];
    const int gy = (r.g >> 10) & 1023, gz = (r.g >> 20) & 1023;
    int j = gz - z;
    if (j < 0) j += K3;
    const int sl = gy / R;
    int nsl = qs + 1;
    if (nsl >= NQ) nsl -= NQ;
    if (j < ORDER && (sl == qs || (sl == nsl && gy - sl * R < ORDER - 1)))
      spread_atom<P, K1, K2, ORDER, R, PITCH>(tile, r, ORDER - 1 - j, y0, scale);
  }
  __syncthreads();
  TRACE(1, 2);

  if (a.keep_grid) {
    Acc* dbg = reinterpret_cast<Acc*>(a.ws + a.lay.dbg) + ((size_t)z * K2 + y0) * K1;
    for (int i = tid; i < R * K1; i += NTS) dbg[i] = tile[(i / K1) * PITCH + (i % K1)];
    __syncthreads();  // the x transform below overwrites the tile in place
  }

  // --- x: real-to-complex, one row per group of fft_lanes(M) lanes.
  constexpr int TM = fft_lanes(M);
  if constexpr (reg_x_ok<K1>()) {
    static_assert(TM == M / 8 && R * TM <= NTS, "register x rows");
    if (tid < R * TM) {
      const int y = tid / TM, j = tid - y * TM;
      cplx<T> v[8];
      if constexpr (P::fixed) {
        // int64 -> FP64 -> FP32: x_{2n} and x_{2n+1} of points n = j + TM r
        const double inv_scale = ldexp(1.0, -a.frac_bits);
        const Acc* ri = tile + y * PITCH;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          const int n = j + TM * r;
          v[r] = {(float)((double)(long long)ri[2 * n] * inv_scale),
                  (float)((double)(long long)ri[2 * n + 1] * inv_scale)};
        }
      } else {
        const cplx<T>* rz = reinterpret_cast<const cplx<T>*>(tile + y * PITCH);
#pragma unroll
        for (int r = 0; r < 8; ++r) v[r] = rz[j + TM * r];
      }
      // X_k of row y straight to column k (runs of R rows per x' across the
      // wavefront's rows)
      typename P::spec* sp = reinterpret_cast<typename P::spec*>(a.ws + a.lay.spec) +
                             (size_t)z * K2 + y0 + y;
      r2c_row_reg<T, K1>(v, reinterpret_cast<cplx<T>*>(tile + y * PITCH), j, xscr + (tid - j) * 9,
                         tw, [&](int k, const cplx<T>& x) { spec_st(&sp[(size_t)k * K3 * K2], x); });
    }
    TRACE(1, 15);
    return;
  } else
  for (int task = tid; task < R * TM; task += NTS) {
    const int y = task / TM, l = task - y * TM;
    cplx<T>* row = reinterpret_cast<cplx<T>*>(tile + y * PITCH);
    if constexpr (P::fixed) {
      // int64 -> float in place: x_j at float slot j, so the row reads as the
      // packed complex sequence z_n = x_{2n} + i x_{2n+1}
      const double inv_scale = ldexp(1.0, -a.frac_bits);
      constexpr int PER = K1 / TM;
      float v[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const long long iv = (long long)tile[y * PITCH + l + i * TM];
        v[i] = (float)((double)iv * inv_scale);
      }
      lds_order();
#pragma unroll
      for (int i = 0; i < PER; ++i) reinterpret_cast<float*>(row)[l + i * TM] = v[i];
      lds_order();
    }
    fft_pencil<T, M, -1>(row, 1, l, tw, 2);
    r2c_post<T, K1>(row, l, tw);
  }
  __syncthreads();
  TRACE(1, 3);

  // half spectrum columns [x'][z][y]: runs of R rows per x'
  using S = typename P::spec;
  S* spec = reinterpret_cast<S*>(a.ws + a.lay.spec) + (size_t)z * K2 + y0;
  constexpr int PC = P::fixed ? PITCH : PITCH / 2;
  const cplx<T>* tc = reinterpret_cast<const cplx<T>*>(tile);
  for (int i = tid; i < R * KH; i += NTS) {
    const int x = i / R, y = i - x * R;
    spec_st(&spec[(size_t)x * K3 * K2 + y], tc[y * PC + x]);
  }
  TRACE(1, 15);
}

// ---------------------------------------------------------------------------
// k_conv: one x' column of the half spectrum (every y and z of one m1) per
// workgroup: forward y and z transforms, the influence function with FP64
// energy/virial partials, inverse z and y transforms (§III.A.2: the slab
// transforms, the multiplication by Green's function data and the inverse
// transforms, with the two corner turns folded into this one column).  When
// the K3 x K2 column does not fit in LDS (FP64, 128^3) it is staged through
// the workspace in halves.
// ---------------------------------------------------------------------------
// Threads per column: 1024, or 512 where the FP64 radix stages of long
// pencils (72 points and up) need more than the 128 registers a 1024-thread
// workgroup leaves per lane.
template <class P, class G>
__host__ __device__ constexpr int conv_threads() {
  return (sizeof(typename P::real) == 8 && (G::K2 >= 72 || G::K3 >= 72)) ? 512 : 1024;
}
// Batched columns (FP32 precisions): 512 threads where that still covers
// every FFT task of a pass (64-point pencils and shorter), so that two
// columns share a CU.
template <class P, class G, bool BATCH>
__host__ __device__ constexpr int conv_block() {
  return (BATCH && P::fixed && conv_threads<P, G>() == 1024 && fft_lanes(G::K2) * G::K3 <= 512 &&
          fft_lanes(G::K3) * G::K2 <= 512)
             ? 512
             : conv_threads<P, G>();
}
template <class P, class G>
__host__ __device__ constexpr size_t conv_tables_bytes() {
  // y and z twiddles, per-axis factors, one energy/virial row per wavefront
  return (size_t)(G::K2 + G::K3) * sizeof(cplx<typename P::real>) +
         (size_t)(G::K1 + G::K2 + G::K3) * sizeof(double) + 16 * 8 * sizeof(double);
}
// Row pitch (complex elements) of the column in LDS: rows are y pencils of
// K points, columns z pencils; chosen with a bank model of the Stockham
// stages over both (64-lane wavefront, 4-byte banks).
template <class P>
__host__ __device__ constexpr int conv_pitch(int K) {
  return sizeof(typename P::real) == 4
             ? (K == 16 ? 18 : K == 32 ? 38 : K == 48 ? 50 : K == 64 ? 71 : K == 96 ? 100
                : K == 128 ? 135 : K + 1)
             : (K == 64 ? 71 : K == 96 ? 102 : K == 128 ? 131 : K + 1);
}
// LDS chunks of the column: 1 when all K3 rows fit, else 2 (halves of the
// z-planes in the y passes, halves of the y rows in the z pass)
template <class P, class G>
__host__ __device__ constexpr int conv_nchunks() {
  return (size_t)G::K3 * conv_pitch<P>(G::K2) * sizeof(cplx<typename P::real>) +
                     conv_tables_bytes<P, G>() <= kMaxLds
             ? 1
             : 2;
}
// z pass row pitch when the column is staged in chunks
template <class P, class G>
__host__ __device__ constexpr int conv_zpitch() {
  return conv_nchunks<P, G>() == 1 ? conv_pitch<P>(G::K2) : G::K2 / 2 + 3;
}
template <class P, class G>
__host__ __device__ constexpr size_t conv_buf_bytes() {
  constexpr size_t NC = conv_nchunks<P, G>();
  constexpr size_t ny = (G::K3 / NC) * conv_pitch<P>(G::K2), nz = (size_t)G::K3 * conv_zpitch<P, G>();
  return (ny > nz ? ny : nz) * sizeof(cplx<typename P::real>);
}
template <class P, class G>
__host__ __device__ constexpr size_t conv_lds_bytes() {
  return conv_buf_bytes<P, G>() + conv_tables_bytes<P, G>();
}

// Per-axis factors T_a(m) = |b_a(m)|^2 exp(-pi^2 mt^2 / (beta L_a)^2) of an
// orthorhombic cell (a general cell keeps the bare moduli: its Gaussian does
// not factor), x then y then z, into bs[K1 + K2 + K3].
template <class G, int NT>
__device__ __forceinline__ void axis_factors(const Args& a, double* bs) {
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  constexpr double PI = 3.14159265358979323846;
  const double* bsg = reinterpret_cast<const double*>(a.ws + a.lay.bsq);
  const double fac = PI * PI / (a.beta * a.beta);
  // (values selected, not a.invL[ax]: a dynamic index, or a select of
  // addresses, would move a batched run's Args copy to scratch)
  const double il0 = a.invL[0], il1 = a.invL[1], il2 = a.invL[2];
  for (int i = threadIdx.x; i < K1 + K2 + K3; i += NT) {
    const int ax = i < K1 ? 0 : i < K1 + K2 ? 1 : 2;
    const int Ka = ax == 0 ? K1 : ax == 1 ? K2 : K3;
    const int m = i - (ax == 0 ? 0 : ax == 1 ? K1 : K1 + K2);
    const int mt = (2 * m <= Ka) ? m : m - Ka;
    const double il = ax == 0 ? il0 : ax == 1 ? il1 : il2;
    const double u = mt * il;
    bs[i] = a.triclinic ? bsg[i] : bsg[i] * exp(-fac * u * u);
  }
}

// The convolution's extra workgroup: keeps the bucket counts of this step
// for the interpolation pass and clears them (and the overflow count) for
// the next step's binning; checks the fixed-point headroom.
template <class P, class G, int NT>
__device__ __forceinline__ void keep_counts(const Args& a, double* wred) {
  const int tid = threadIdx.x;
  unsigned* bcnt = reinterpret_cast<unsigned*>(a.ws + a.lay.bcnt);
  unsigned* bcnt2 = reinterpret_cast<unsigned*>(a.ws + a.lay.bcnt2);
  unsigned* ovf = reinterpret_cast<unsigned*>(a.ws + a.lay.ovf);
  constexpr int NBINS = 2 * G::K3 * nq_of(G::K2, P::fixed);
  for (int b = tid; b < NBINS; b += NT) {
    bcnt2[b] = bcnt[b];
    bcnt[b] = 0u;
  }
  if (tid == 0) {
    ovf[1] = ovf[0];
    ovf[0] = 0u;
  }
  if constexpr (P::fixed) {
    // sum |q| 2^F must stay below 2^51 so that every contribution and grid
    // value is exact in FP64 and the rounding of to_fixed holds
    const double* absq = reinterpret_cast<const double*>(a.ws + a.lay.absq);
    double v[1] = {0.0};
    for (int c = tid; c < a.n_chunks; c += NT) v[0] += absq[c];
    block_sums<1>(v, wred);
    if (tid == 15 && v[0] * ldexp(1.0, a.frac_bits) >= 2251799813685248.0)
      atomicOr(reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl), PME_FLAG_OVERFLOW);
  }
}

// Influence function on z-transformed modes of column x' = xp held in LDS as
// buf[z * PZ + yy] (z < K3, y = y0 + yy, yy < CY): the modes of virtual
// thread vt of VT (mode i = vt + k VT) are multiplied by G(m) and their
// energy/virial terms are added to acc.  The partition over virtual threads,
// not the launch's thread count, fixes the order of every sum.
// G(m) = c B(m) exp(-pi^2 |m|^2 / beta^2) / (pi V |m|^2) with
// B exp(-pi^2|m|^2/beta^2) = T_x(m1) T_y(m2) T_z(m3) in an orthorhombic
// cell.  The half spectrum counts every m1 = 1 .. K1/2-1 twice (its
// Hermitian partner), m1 = 0 and m1 = K1/2 once.  Per mode, with
// e = w G |F|^2 and u = 1/|m|^2 + pi^2/beta^2:
//   E += e,  P_ab += e (delta_ab - 2 u m_a m_b),
// accumulated as S0 = sum e and S_ab = sum e u m_a m_b (acc: S0, Sxx, Syy,
// Szz, Sxy, Sxz, Syz), so that P_aa = S0 - 2 S_aa and P_ab = -2 S_ab.  A
// Nyquist index aliases +K_a/2 and -K_a/2 equally, so its sign-odd
// (off-diagonal) products vanish.
// Constants of one x' column for the influence function.
struct InflCol {
  double fac, mvx, nx, wx, mvx2, A;
};
template <class G>
__device__ __forceinline__ InflCol infl_col(const Args& a, int xp, const double* bs) {
  constexpr double PI = 3.14159265358979323846;
  InflCol c;
  const double pref = a.coulomb / (PI * a.volume);
  c.fac = PI * PI / (a.beta * a.beta);
  c.mvx = xp * a.invL[0];
  c.nx = (2 * xp == G::K1) ? 0.0 : c.mvx;
  c.wx = (xp == 0 || 2 * xp == G::K1) ? 0.5 : 1.0;
  c.mvx2 = c.mvx * c.mvx;
  c.A = pref * bs[xp];
  return c;
}

// One mode (xp, y, z) of an orthorhombic cell: returns G(m) F(m) and adds
// the mode's energy/virial terms to acc.
template <class G, typename T>
__device__ __forceinline__ cplx<T> infl_ortho(const Args& a, const InflCol& c, int xp, int y,
                                              int z, const double* bs, cplx<T> f, double* acc) {
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  const int my = (2 * y <= K2) ? y : y - K2, mz = (2 * z <= K3) ? z : z - K3;
  const double mvy = my * a.invL[1], mvz = mz * a.invL[2];
  const double ny = (2 * y == K2) ? 0.0 : mvy, nz = (2 * z == K3) ? 0.0 : mvz;
  // m = 0 carries no energy (G(0) = 0): its |m|^2 is replaced by 1 and its
  // G by 0, without a branch
  const bool m0 = (xp == 0) && (y == 0) && (z == 0);
  const double msq = m0 ? 1.0 : fma(mvz, mvz, fma(mvy, mvy, c.mvx2));
  // 1/msq: hardware reciprocal and two Newton steps
  double r = __builtin_amdgcn_rcp(msq);
  r = fma(r, fma(-msq, r, 1.0), r);
  r = fma(r, fma(-msq, r, 1.0), r);
  const double gm = m0 ? 0.0 : c.A * bs[K1 + y] * bs[K1 + K2 + z] * r;  // G(m)
  const double f2 = fma((double)f.x, (double)f.x, (double)f.y * (double)f.y);
  const double e = c.wx * gm * f2;
  const double eu = e * (r + c.fac);
  const double eux = eu * c.mvx, euy = eu * mvy, eun = eu * c.nx;
  acc[0] += e;
  acc[1] = fma(eux, c.mvx, acc[1]);
  acc[2] = fma(euy, mvy, acc[2]);
  acc[3] = fma(eu * mvz, mvz, acc[3]);
  acc[4] = fma(eun, ny, acc[4]);
  acc[5] = fma(eun, nz, acc[5]);
  acc[6] = fma(eu * ny, nz, acc[6]);
  const T g = (T)gm;
  return {f.x * g, f.y * g};
}

// One mode of a general cell: m = m1 a*_1 + m2 a*_2 + m3 a*_3 does not
// separate; each Nyquist index is averaged over its two signs explicitly.
template <class G, typename T>
__device__ __forceinline__ cplx<T> infl_general(const Args& a, const InflCol& c, int xp, int y,
                                                int z, const double* bs, cplx<T> f, double* acc) {
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  const int ms0[3] = {xp, (2 * y <= K2) ? y : y - K2, (2 * z <= K3) ? z : z - K3};
  const int ny3[3] = {2 * xp == K1, 2 * y == K2, 2 * z == K3};
  const int nvar = 1 << (ny3[0] + ny3[1] + ny3[2]);
  const double f2 = fma((double)f.x, (double)f.x, (double)f.y * (double)f.y);
  double gm = 0.0;  // G(m), averaged over the Nyquist signs
  if (xp != 0 || y != 0 || z != 0) {
    const double Bw = c.A * bs[K1 + y] * bs[K1 + K2 + z] / nvar;
    for (int v = 0; v < nvar; ++v) {
      double ms[3];
      int bit = 0;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        ms[ax] = ms0[ax];
        if (ny3[ax]) {
          if ((v >> bit) & 1) ms[ax] = -ms[ax];
          ++bit;
        }
      }
      double mv[3];
#pragma unroll
      for (int c2 = 0; c2 < 3; ++c2)
        mv[c2] = ms[0] * a.rec[c2] + ms[1] * a.rec[3 + c2] + ms[2] * a.rec[6 + c2];
      const double msq = mv[0] * mv[0] + mv[1] * mv[1] + mv[2] * mv[2];
      double r = __builtin_amdgcn_rcp(msq);
      r = fma(r, fma(-msq, r, 1.0), r);
      r = fma(r, fma(-msq, r, 1.0), r);
      const double Gv = Bw * exp(-c.fac * msq) * r;
      const double e = c.wx * Gv * f2;
      const double eu = e * (r + c.fac);
      acc[0] += e;
      acc[1] = fma(eu * mv[0], mv[0], acc[1]);
      acc[2] = fma(eu * mv[1], mv[1], acc[2]);
      acc[3] = fma(eu * mv[2], mv[2], acc[3]);
      acc[4] = fma(eu * mv[0], mv[1], acc[4]);
      acc[5] = fma(eu * mv[0], mv[2], acc[5]);
      acc[6] = fma(eu * mv[1], mv[2], acc[6]);
      gm += Gv;
    }
  }
  const T g = (T)gm;
  return {f.x * g, f.y * g};
}

template <class P, class G, int CY, int PZ, int VT>
__device__ __forceinline__ void influence(const Args& a, cplx<typename P::real>* buf, int xp,
                                          int y0, const double* bs, double* acc, int vt) {
  constexpr int K3 = G::K3;
  const InflCol c = infl_col<G>(a, xp, bs);
  if (a.triclinic) {
    for (int i = vt; i < K3 * CY; i += VT) {
      const int z = i / CY, yy = i - z * CY;
      buf[z * PZ + yy] = infl_general<G>(a, c, xp, y0 + yy, z, bs, buf[z * PZ + yy], acc);
    }
  } else {
    constexpr int NIT = (K3 * CY + VT - 1) / VT;
    constexpr int UNR = NIT <= 4 ? NIT : 2;
#pragma unroll UNR
    for (int it = 0; it < NIT; ++it) {
      const int i = vt + it * VT;
      if ((K3 * CY) % VT != 0 && i >= K3 * CY) break;
      const int z = i / CY, yy = i - z * CY;
      buf[z * PZ + yy] = infl_ortho<G>(a, c, xp, y0 + yy, z, bs, buf[z * PZ + yy], acc);
    }
  }
}

// Energy/virial: a fixed-order DPP sum over the wavefront, one partial row
// (E, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz) written at row `r`, the rows added in
// row order later.
__device__ __forceinline__ void ev_row(const Args& a, double* acc, int r) {
  wave_sums<7>(acc);
  if ((threadIdx.x & 63) == 63) {
    double* row = reinterpret_cast<double*>(a.ws + a.lay.partial) + r * 8;
    row[0] = acc[0];
#pragma unroll
    for (int c = 1; c < 4; ++c) row[c] = acc[0] - 2.0 * acc[c];
#pragma unroll
    for (int c = 4; c < 7; ++c) row[c] = -2.0 * acc[c];
  }
}

template <class P, class G, bool BATCH>
__global__ __launch_bounds__((conv_block<P, G, BATCH>()),
                             (conv_block<P, G, BATCH>() == 512 ? 4 : 1)) void k_conv(Args a_in,
                                                                                      BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  constexpr int KH = K1 / 2 + 1;
  constexpr int NC = conv_nchunks<P, G>();
  constexpr int CZ = K3 / NC;                  // z-planes per chunk (y passes)
  constexpr int CY = K2 / NC;                  // y rows per chunk (z pass)
  constexpr int PY = conv_pitch<P>(K2);        // y pass: one row of pitch PY per z
  constexpr int PZ = conv_zpitch<P, G>();      // z pass: one row of pitch PZ per z
  constexpr int TY = fft_lanes(K2), TZ = fft_lanes(K3);
  constexpr int NT = conv_block<P, G, BATCH>();
  // the modes are dealt to VT virtual threads, NV per thread, as a VT-thread
  // launch deals them, so that batched and single steps add alike
  constexpr int VT = conv_threads<P, G>(), NV = VT / NT;
  constexpr bool EARLY_EV = NV > 1 && NC == 1;
  static_assert(conv_lds_bytes<P, G>() <= kMaxLds, "convolution column does not fit in LDS");
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* twy = reinterpret_cast<cplx<T>*>(smem + conv_buf_bytes<P, G>());
  cplx<T>* twz = twy + K2;
  double* bs = reinterpret_cast<double*>(twz + K3);  // x, y, z factors
  double* wred = bs + K1 + K2 + K3;
  TRACE(2, 0);
  const int tid = threadIdx.x;
  if (blockIdx.x == KH) {
    keep_counts<P, G, NT>(a, wred);
    return;
  }
  const int xp = blockIdx.x;  // m1
  using S = typename P::spec;
  S* col = reinterpret_cast<S*>(a.ws + a.lay.spec) + (size_t)xp * K3 * K2;  // [z][y]
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  // the first chunk's loads are issued before the tables are computed
  // (when they fit in a few registers)
  constexpr int EPT = (CZ * K2 + NT - 1) / NT;
  constexpr bool PREFETCH = P::fixed && EPT * sizeof(cplx<T>) <= 32;
  cplx<T> first[PREFETCH ? EPT : 1];
  if constexpr (PREFETCH) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int i = min(tid + k * NT, CZ * K2 - 1);
      first[k] = spec_ld(&col[i]);
    }
  }
  // the y and z twiddle tables follow the x table
  for (int i = tid; i < K2 + K3; i += NT) twy[i] = twg[K1 + i];
  axis_factors<G, NT>(a, bs);

  // --- forward y: one pencil per z
  for (int c = 0; c < NC; ++c) {
    const int z0 = c * CZ;
    if constexpr (PREFETCH) {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const int i = tid + k * NT;
        if (i < CZ * K2) buf[(i / K2) * PY + (i % K2)] = first[k];
      }
    } else {
      for (int i = tid; i < CZ * K2; i += NT) {
        const int zz = i / K2, y = i - zz * K2;
        buf[zz * PY + y] = spec_ld(&col[(size_t)(z0 + zz) * K2 + y]);
      }
    }
    __syncthreads();
    for (int task = tid; task < CZ * TY; task += NT) {
      const int zz = task / TY, l = task - zz * TY;
      fft_pencil<T, K2, -1>(buf + zz * PY, 1, l, twy, 1);
    }
    __syncthreads();
    if constexpr (NC > 1) {
      for (int i = tid; i < CZ * K2; i += NT) {
        const int zz = i / K2, y = i - zz * K2;
        spec_st(&col[(size_t)(z0 + zz) * K2 + y], buf[zz * PY + y]);
      }
      __syncthreads();
    }
  }
  TRACE(2, 1);

  // --- z: forward transform, influence function, inverse transform
  double acc[NV][7];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int c = 0; c < 7; ++c) acc[v][c] = 0.0;
  for (int c = 0; c < NC; ++c) {
    const int y0 = c * CY;
    if constexpr (NC > 1) {
      for (int i = tid; i < K3 * CY; i += NT) {
        const int z = i / CY, yy = i - z * CY;
        buf[z * PZ + yy] = spec_ld(&col[(size_t)z * K2 + y0 + yy]);
      }
      __syncthreads();
    }
    for (int task = tid; task < CY * TZ; task += NT) {
      const int yy = task / TZ, l = task - yy * TZ;
      fft_pencil<T, K3, -1>(buf + yy, PZ, l, twz, 1);
    }
    __syncthreads();
    TRACE(2, 2);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      influence<P, G, CY, PZ, VT>(a, buf, xp, y0, bs, acc[v], tid + v * NT);
      // (one virtual thread's sums written before the next one's start)
      if constexpr (EARLY_EV) ev_row(a, acc[v], xp * (VT / 64) + ((tid + v * NT) >> 6));
    }
    __syncthreads();
    TRACE(2, 3);
    for (int task = tid; task < CY * TZ; task += NT) {
      const int yy = task / TZ, l = task - yy * TZ;
      fft_pencil<T, K3, 1>(buf + yy, PZ, l, twz, 1);
    }
    __syncthreads();
    if constexpr (NC > 1) {
      for (int i = tid; i < K3 * CY; i += NT) {
        const int z = i / CY, yy = i - z * CY;
        spec_st(&col[(size_t)z * K2 + y0 + yy], buf[z * PZ + yy]);
      }
      __syncthreads();
    }
  }
  TRACE(2, 5);

  // --- inverse y
  for (int c = 0; c < NC; ++c) {
    const int z0 = c * CZ;
    if constexpr (NC > 1) {
      for (int i = tid; i < CZ * K2; i += NT) {
        const int zz = i / K2, y = i - zz * K2;
        buf[zz * PY + y] = spec_ld(&col[(size_t)(z0 + zz) * K2 + y]);
      }
      __syncthreads();
    }
    for (int task = tid; task < CZ * TY; task += NT) {
      const int zz = task / TY, l = task - zz * TY;
      fft_pencil<T, K2, 1>(buf + zz * PY, 1, l, twy, 1);
    }
    __syncthreads();
    for (int i = tid; i < CZ * K2; i += NT) {
      const int zz = i / K2, y = i - zz * K2;
      spec_st(&col[(size_t)(z0 + zz) * K2 + y], buf[zz * PY + y]);
    }
    if constexpr (NC > 1) __syncthreads();
  }
  // placed after the last stores so that it overlaps their completion
  // (unless the registers it holds are needed for occupancy)
  if constexpr (!EARLY_EV) {
#pragma unroll
    for (int v = 0; v < NV; ++v) ev_row(a, acc[v], xp * (VT / 64) + ((tid + v * NT) >> 6));
  }
  TRACE(2, 15);
}

// ---------------------------------------------------------------------------
// Split convolution (the default for large columns, K2 K3 >= 8192, e.g.
// 128^3, where one workgroup per x' column leaves most of the chip idle and
// makes the FP64 influence function a one-CU job): three launches of small
// workgroups, with the half spectrum in the workspace between them --
//   k_conv_y<-1>  forward y transforms of a chunk of z-rows of one column
//   k_conv_z      z transforms, influence function and inverse z transforms
//                 of a chunk of y-columns of one column (plus the counts
//                 workgroup)
//   k_conv_y<+1>  inverse y transforms
// ---------------------------------------------------------------------------
constexpr int kPassThreads = 256;
template <class G>
__host__ __device__ constexpr int pass_cz() {  // z-rows per y-pass workgroup
  return kPassThreads / fft_lanes(G::K2);
}
template <class G>
__host__ __device__ constexpr int pass_cy() {  // y-columns per z-pass workgroup
  return kPassThreads / fft_lanes(G::K3);
}
template <class P, class G>
__host__ __device__ constexpr size_t conv_y_lds_bytes() {
  return ((size_t)pass_cz<G>() * conv_pitch<P>(G::K2) + G::K2) * sizeof(cplx<typename P::real>);
}
template <class P, class G>
__host__ __device__ constexpr size_t conv_z_lds_bytes() {
  return ((size_t)G::K3 * (pass_cy<G>() + 1) + G::K3) * sizeof(cplx<typename P::real>) +
         (size_t)(G::K1 + G::K2 + G::K3) * sizeof(double) + 16 * 8 * sizeof(double);
}

// (the forward pass reads the spectrum and writes the full-precision
// intermediate; the inverse pass the other way round; the two are one
// region unless the spectrum is kept in binary16)
template <class P, class G, int DIR, bool BATCH>
__global__ __launch_bounds__(kPassThreads) void k_conv_y(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  using S = typename P::spec;
  using M = cplx<T>;
  using In = std::conditional_t<(DIR < 0), S, M>;
  using Out = std::conditional_t<(DIR < 0), M, S>;
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  constexpr int CZ = pass_cz<G>(), NZC = K3 / CZ;
  constexpr int PY = conv_pitch<P>(K2), TY = fft_lanes(K2);
  static_assert(K3 % CZ == 0 && CZ * TY == kPassThreads, "y pass chunks do not tile the column");
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + CZ * PY;
  const int tid = threadIdx.x;
  const int xp = blockIdx.x / NZC, z0 = (blockIdx.x - xp * NZC) * CZ;
  const size_t off = ((size_t)xp * K3 + z0) * K2;  // rows [zz][y]
  const In* src = reinterpret_cast<const In*>(a.ws + (DIR < 0 ? a.lay.spec : a.lay.mid)) + off;
  Out* dst = reinterpret_cast<Out*>(a.ws + (DIR < 0 ? a.lay.mid : a.lay.spec)) + off;
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < CZ * K2; i += kPassThreads) {
    const int zz = i / K2, y = i - zz * K2;
    buf[zz * PY + y] = spec_ld(&src[i]);
  }
  for (int i = tid; i < K2; i += kPassThreads) tw[i] = twg[K1 + i];
  __syncthreads();
  {
    const int zz = tid / TY, l = tid - zz * TY;
    fft_pencil<T, K2, DIR>(buf + zz * PY, 1, l, tw, 1);
  }
  __syncthreads();
  for (int i = tid; i < CZ * K2; i += kPassThreads) {
    const int zz = i / K2, y = i - zz * K2;
    spec_st(&dst[i], buf[zz * PY + y]);
  }
}

template <class P, class G, bool BATCH>
__global__ __launch_bounds__(kPassThreads) void k_conv_z(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3, KH = K1 / 2 + 1;
  constexpr int CY = pass_cy<G>(), NYC = K2 / CY, PZ = CY + 1, TZ = fft_lanes(K3);
  constexpr int NT = kPassThreads;
  static_assert(K2 % CY == 0 && CY * TZ == NT, "z pass chunks do not tile the column");
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + K3 * PZ;
  double* bs = reinterpret_cast<double*>(tw + K3);  // x, y, z factors
  double* wred = bs + K1 + K2 + K3;
  const int tid = threadIdx.x;
  TRACE(4, 0);
  if (blockIdx.x == KH * NYC) {
    keep_counts<P, G, NT>(a, wred);
    return;
  }
  const int xp = blockIdx.x / NYC, y0 = (blockIdx.x - xp * NYC) * CY;
  cplx<T>* col = reinterpret_cast<cplx<T>*>(a.ws + a.lay.mid) + (size_t)xp * K3 * K2;  // [z][y]
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < K3 * CY; i += NT) {
    const int z = i / CY, yy = i - z * CY;
    buf[z * PZ + yy] = spec_ld(&col[(size_t)z * K2 + y0 + yy]);
  }
  for (int i = tid; i < K3; i += NT) tw[i] = twg[K1 + K2 + i];
  axis_factors<G, NT>(a, bs);
  __syncthreads();
  TRACE(4, 1);
  const int yy = tid / TZ, l = tid - yy * TZ;
  fft_pencil<T, K3, -1>(buf + yy, PZ, l, tw, 1);
  __syncthreads();
  TRACE(4, 2);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  influence<P, G, CY, PZ, NT>(a, buf, xp, y0, bs, acc, tid);
  __syncthreads();
  TRACE(4, 3);
  fft_pencil<T, K3, 1>(buf + yy, PZ, l, tw, 1);
  __syncthreads();
  TRACE(4, 4);
  for (int i = tid; i < K3 * CY; i += NT) {
    const int z = i / CY, yy2 = i - z * CY;
    spec_st(&col[(size_t)z * K2 + y0 + yy2], buf[z * PZ + yy2]);
  }
  ev_row(a, acc, blockIdx.x * (NT / 64) + (tid >> 6));
  TRACE(4, 15);
}

// ---------------------------------------------------------------------------
// k_conv_reg: the column convolution with register-resident transforms
// (y and z pencils of 32 or 64 points; FP32 or FP64).  A pencil of
// N = 8 R points is held by R lanes of one wavefront, 8 values per lane
// (lane j holds points j + R r): a radix-8 DFT over r in registers, the
// twiddles W_N^(j s), an R x 8 transpose through the wavefront's own LDS
// scratch, then radix-R DFTs over the lanes in registers (Cooley-Tukey with
// N = 8 R), which leaves lane j with the modes jE + e + 8t (E = 8/R, e < E,
// t < R).  The inverse runs the same steps backwards from that layout.  The
// forward z transform, the influence function and the inverse z transform
// work on the same registers, so LDS carries only the two corner turns and
// the transposes (the one-workgroup column of k_conv moves every element
// through LDS twice per radix stage).  One workgroup per x' column.
// ---------------------------------------------------------------------------
template <class G>
__host__ __device__ constexpr bool conv_reg_shape() {
  return (G::K2 == 32 || G::K2 == 64) && (G::K3 == 32 || G::K3 == 64);
}
template <class G>
__host__ __device__ constexpr int conv_reg_threads() {  // pencils x lanes, either pass
  return G::K2 * G::K3 / 8;
}
template <class G>
__host__ __device__ constexpr int conv_reg_pitch() {  // column row pitch (complex)
  return G::K2 + 8;
}
template <class P, class G>
__host__ __device__ constexpr size_t conv_reg_lds_bytes() {
  // the column, then the transposes' scratch (a row of 8 values, pitch 9, per
  // lane), then the y and z twiddles
  return ((size_t)G::K3 * conv_reg_pitch<G>() + (size_t)conv_reg_threads<G>() * 9 + G::K2 +
          G::K3) * sizeof(cplx<typename P::real>) +
         (size_t)(G::K1 + G::K2 + G::K3) * sizeof(double) + 16 * 8 * sizeof(double);
}

template <class P, class G, bool BATCH>
__global__ __launch_bounds__(conv_reg_threads<G>()) void k_conv_reg(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  using S = typename P::spec;
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3, KH = K1 / 2 + 1;
  constexpr int NT = conv_reg_threads<G>(), PB = conv_reg_pitch<G>();
  constexpr int RY = K2 / 8, EY = 8 / RY, RZ = K3 / 8, EZ = 8 / RZ;
  static_assert(conv_reg_shape<G>(), "register transforms: 32 or 64 points");
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);         // [z][y], pitch PB
  cplx<T>* scr0 = buf + K3 * PB;                            // transposes: 9 per lane
  cplx<T>* twy = scr0 + NT * 9;
  cplx<T>* twz = twy + K2;
  double* bs = reinterpret_cast<double*>(twz + K3);         // x, y, z factors
  double* wred = bs + K1 + K2 + K3;
  const int tid = threadIdx.x;
  TRACE(2, 0);
  if (blockIdx.x == KH) {
    keep_counts<P, G, NT>(a, wred);
    return;
  }
  const int xp = blockIdx.x;  // m1
  S* col = reinterpret_cast<S*>(a.ws + a.lay.spec) + (size_t)xp * K3 * K2;  // [z][y]
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);

  // --- forward y: pencil z = tid / RY, lane j loads points j + RY r
  cplx<T> v[8];
  {
    const int z = tid / RY, j = tid - z * RY;
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = spec_ld(&col[(size_t)z * K2 + j + RY * r]);
  }
  for (int i = tid; i < K2 + K3; i += NT) twy[i] = twg[K1 + i];
  axis_factors<G, NT>(a, bs);
  __syncthreads();
  TRACE(2, 1);
  // each lane's twiddles for both directions (shared by the two passes when
  // the y and z pencils have one length)
  RegTw<T, K2> wy;
  wy.load(tid % RY, twy);
  RegTw<T, K3> wz_own;
  if constexpr (K2 != K3) wz_own.load(tid % RZ, twz);
  const RegTw<T, K3>& wz = [&]() -> const RegTw<T, K3>& {
    if constexpr (K2 == K3) return wy;
    else return wz_own;
  }();
  {
    const int z = tid / RY, j = tid - z * RY;
    rfft_fwd<T, K2, -1>(v, j, scr0 + (tid - j) * 9, wy);
#pragma unroll
    for (int e = 0; e < EY; ++e)
#pragma unroll
      for (int t = 0; t < RY; ++t) buf[z * PB + j * EY + e + 8 * t] = v[e * RY + t];
  }
  __syncthreads();
  TRACE(2, 2);

  // --- z: forward transform, influence function, inverse transform
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  {
    const int y = tid / RZ, j = tid - y * RZ;
#pragma unroll
    for (int r = 0; r < 8; ++r) v[r] = buf[(j + RZ * r) * PB + y];
    rfft_fwd<T, K3, -1>(v, j, scr0 + (tid - j) * 9, wz);
    const InflCol c = infl_col<G>(a, xp, bs);
    if (a.triclinic) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int z = j * EZ + k / RZ + 8 * (k % RZ);
        v[k] = infl_general<G>(a, c, xp, y, z, bs, v[k], acc);
      }
    } else {
      // orthorhombic: the lane's modes share m1 and m2, so the factors of
      // x and y are taken once per lane and the virial sums are kept as
      // S0 = sum e, Su = sum eu, Sz = sum eu nz, Szz = sum eu mz^2, from
      // which P_xx, P_yy, P_xy (m1^2 Su, m2^2 Su, n1 n2 Su) and P_xz, P_yz
      // (n1 Sz, n2 Sz) follow
      const int my = (2 * y <= K2) ? y : y - K2;
      const double mvy = my * a.invL[1], ny = (2 * y == K2) ? 0.0 : mvy;
      const double Ay = c.A * bs[K1 + y], base = fma(mvy, mvy, c.mvx2);
      double s0 = 0.0, su = 0.0, sz = 0.0, szz = 0.0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const int z = j * EZ + k / RZ + 8 * (k % RZ);
        const int mz = (2 * z <= K3) ? z : z - K3;
        const double mvz = mz * a.invL[2], nz = (2 * z == K3) ? 0.0 : mvz;
        const bool m0 = (xp == 0) && (y == 0) && (z == 0);
        const double msq = m0 ? 1.0 : fma(mvz, mvz, base);
        double r = __builtin_amdgcn_rcp(msq);
        r = fma(r, fma(-msq, r, 1.0), r);
        r = fma(r, fma(-msq, r, 1.0), r);
        const double gm = m0 ? 0.0 : Ay * bs[K1 + K2 + z] * r;  // G(m)
        const double f2 = fma((double)v[k].x, (double)v[k].x, (double)v[k].y * (double)v[k].y);
        const double e = c.wx * gm * f2;
        const double eu = e * (r + c.fac);
        s0 += e;
        su += eu;
        sz = fma(eu, nz, sz);
        szz = fma(eu * mvz, mvz, szz);
        const T g = (T)gm;
        v[k] = {v[k].x * g, v[k].y * g};
      }
      acc[0] = s0;
      acc[1] = c.mvx2 * su;
      acc[2] = (mvy * mvy) * su;
      acc[3] = szz;
      acc[4] = (c.nx * ny) * su;
      acc[5] = c.nx * sz;
      acc[6] = ny * sz;
    }
    rfft_inv<T, K3, 1>(v, j, scr0 + (tid - j) * 9, wz);
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[(j + RZ * r) * PB + y] = v[r];
  }
  // the wavefront's energy/virial row, while the others finish their z pass
  ev_row(a, acc, xp * (NT / 64) + (tid >> 6));
  __syncthreads();
  TRACE(2, 3);

  // --- inverse y, stored back to the column
  {
    const int z = tid / RY, j = tid - z * RY;
#pragma unroll
    for (int e = 0; e < EY; ++e)
#pragma unroll
      for (int t = 0; t < RY; ++t) v[e * RY + t] = buf[z * PB + j * EY + e + 8 * t];
    rfft_inv<T, K2, 1>(v, j, scr0 + (tid - j) * 9, wy);
#pragma unroll
    for (int r = 0; r < 8; ++r) spec_st(&col[(size_t)z * K2 + j + RY * r], v[r]);
  }
  TRACE(2, 15);
}

// Sum of the energy/virial partial rows the step's convolution variant wrote,
// in a fixed order, by the first wavefront of the calling workgroup
// (whatever its size): lane l adds rows l, l+64, ..., then a DPP sum over
// the lanes.
static __device__ void reduce_ev(const Args& a) {
  if (threadIdx.x >= 64) return;
  const double* partial = reinterpret_cast<const double*>(a.ws + a.lay.partial);
  double v[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int r = threadIdx.x; r < a.ev_rows; r += 64) {
#pragma unroll
    for (int c = 0; c < 7; ++c) v[c] += partial[r * 8 + c];
  }
  wave_sums<7>(v);
  if (threadIdx.x == 63) {
#pragma unroll
    for (int c = 0; c < 7; ++c) a.ev[c] = v[c];
  }
}

// ---------------------------------------------------------------------------
// k_inv_x: complex-to-real x transform of one z-plane into the potential
// rows of the workspace (with a (p-1)-point wrap halo in front).  Used on
// large grids before k_interp_phi, and for the debug copy of the potential.
// ---------------------------------------------------------------------------
// Row pitch (complex) of the potential rows of k_inv_x and k_interp: the
// half spectrum X_0 .. X_{K1/2} plus one, widened where the register
// inverse x transform uses the row itself as its transpose scratch (RX
// lanes of 9 complex each).
template <int K1>
__host__ __device__ constexpr int x_row_pitch() {
  return reg_x_ok<K1>() && (K1 / 16) * 9 > K1 / 2 + 2 ? (K1 / 16) * 9 : K1 / 2 + 2;
}
template <class P, class G, int ORDER>
__host__ __device__ constexpr size_t inv_x_lds_bytes() {
  return (size_t)G::K2 * x_row_pitch<G::K1>() * sizeof(cplx<typename P::real>) +
         (size_t)G::K1 * sizeof(cplx<typename P::real>);
}
template <class P, class G, int ORDER>
__host__ __device__ constexpr bool x_inv_reg();  // both interpolations alike

template <class P, class G, int ORDER, bool BATCH>
__global__ __launch_bounds__(kPlaneThreads) void k_inv_x(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  constexpr int M = K1 / 2, KH = K1 / 2 + 1, PC = x_row_pitch<K1>();
  constexpr int PP = phi_pitch_of(K1, ORDER);
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = pl + K2 * PC;
  const int tid = threadIdx.x;
  // (the XCD remap needs a multiple of 8 planes)
  const int z = K3 % kXcds == 0 ? xcd_local(blockIdx.x, K3) : (int)blockIdx.x;
  const typename P::spec* spec = reinterpret_cast<const typename P::spec*>(a.ws + a.lay.spec);
  for (int i = tid; i < KH * K2; i += kPlaneThreads) {
    const int x = i / K2, y = i - x * K2;
    pl[y * PC + x] = spec_ld(&spec[((size_t)x * K3 + z) * K2 + y]);
  }
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < K1; i += kPlaneThreads) tw[i] = twg[i];
  __syncthreads();
  constexpr int TM = fft_lanes(M);
  if constexpr (x_inv_reg<P, G, ORDER>()) {
    for (int task = tid; task < K2 * TM; task += kPlaneThreads) {
      const int y = task / TM, l = task - y * TM;
      c2r_row_reg<T, K1>(pl + y * PC, l, pl + y * PC, tw);  // the row is its scratch
    }
  } else {
    for (int task = tid; task < K2 * TM; task += kPlaneThreads) {
      const int y = task / TM, l = task - y * TM;
      cplx<T>* row = pl + y * PC;
      c2r_pre<T, K1>(row, l, tw);
      fft_pencil<T, M, 1>(row, 1, l, tw, 2);
    }
  }
  __syncthreads();
  T* phi = reinterpret_cast<T*>(a.ws + a.lay.phi) + (size_t)z * K2 * PP;
  for (int i = tid; i < K2 * PP; i += kPlaneThreads) {
    const int y = i / PP, xh = i - y * PP;
    int x = xh - (ORDER - 1);
    if (x < 0) x += K1;
    if (x >= K1) x -= K1;
    phi[i] = reinterpret_cast<const T*>(pl + y * PC)[x];
  }
}

// ---------------------------------------------------------------------------
// k_interp: complex-to-real x transforms and force interpolation for the
// atoms of one (z-plane, y-slice) bin per workgroup (§III.A.3).  The
// workgroup transforms the p planes z-p+1 .. z, rows y0-p+1 .. y0+R-1, of
// the spectrum into LDS -- the potential every atom of the bin reads -- and
// interpolates those atoms from LDS, one per thread; forces go to the
// caller's atom order.
// ---------------------------------------------------------------------------
template <class P, class G, int ORDER>
__host__ __device__ constexpr size_t interp_lds_bytes() {
  constexpr size_t R = G::K2 / nq_of(G::K2, P::fixed), NROW = (size_t)ORDER * (R + ORDER - 1);
  return NROW * x_row_pitch<G::K1>() * sizeof(cplx<typename P::real>) +
         (size_t)G::K1 * sizeof(cplx<typename P::real>) + 4 * sizeof(int);
}
// The register inverse x transform wherever both interpolations have it, so
// that the fused and the split interpolation stay bit-identical.
template <class P, class G, int ORDER>
__host__ __device__ constexpr bool x_inv_reg() {
  return reg_x_ok<G::K1>() && interp_lds_bytes<P, G, ORDER>() <= kMaxLds &&
         inv_x_lds_bytes<P, G, ORDER>() <= kMaxLds;
}

// Force on one atom from the potential: rows(jz, jy) points at the potential
// row of support point (jz, jy) and xs[jx] at the x index of point jx.
template <class P, int ORDER, class Rows>
__device__ __forceinline__ void interpolate(const Args& a, const typename P::rec& r, Rows rows,
                                            const int* xs) {
  using T = typename P::real;
  const double qi = r.qd;
  T thx[ORDER], thy[ORDER], thz[ORDER], dthx[ORDER], dthy[ORDER], dthz[ORDER];
  bspline<ORDER>(r.w[0], thx, dthx);
  bspline<ORDER>(r.w[1], thy, dthy);
  bspline<ORDER>(r.w[2], thz, dthz);
  T sx = 0, sy = 0, sz = 0;
#pragma unroll
  for (int jz = 0; jz < ORDER; ++jz) {
#pragma unroll
    for (int jy = 0; jy < ORDER; ++jy) {
      const T* row = rows(jz, jy);
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int jx = 0; jx < ORDER; ++jx) {
        const T v = row[xs[jx]];
        s0 += thx[jx] * v;
        s1 += dthx[jx] * v;
      }
      sx += thy[jy] * thz[jz] * s1;
      sy += dthy[jy] * thz[jz] * s0;
      sz += thy[jy] * dthz[jz] * s0;
    }
  }
  // derivatives with respect to the scaled coordinates u_a = K_a s_a
  const double d1 = (double)a.K1 * (double)sx, d2 = (double)a.K2 * (double)sy,
               d3 = (double)a.K3 * (double)sz;
  double f[3];
  if (!a.triclinic) {
    f[0] = -qi * (d1 * a.invL[0]);
    f[1] = -qi * (d2 * a.invL[1]);
    f[2] = -qi * (d3 * a.invL[2]);
  } else {
    // F = -q (K_1 s_1 a*_1 + K_2 s_2 a*_2 + K_3 s_3 a*_3)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      f[c] = -qi * (d1 * a.rec[c] + d2 * a.rec[3 + c] + d3 * a.rec[6 + c]);
  }
  double* out = a.forces + 3 * (size_t)r.idx;
  if (a.accumulate) {
    out[0] += f[0];
    out[1] += f[1];
    out[2] += f[2];
  } else {
    out[0] = f[0];
    out[1] = f[1];
    out[2] = f[2];
  }
}

template <class P, class G, int ORDER, bool BATCH>
__global__ __launch_bounds__(kInterpThreads) void k_interp(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  using Rec = typename P::rec;
  constexpr int K1 = G::K1, K2 = G::K2, K3 = G::K3;
  constexpr int M = K1 / 2, KH = M + 1, PC = x_row_pitch<K1>();
  constexpr int NQ = nq_of(K2, P::fixed), R = K2 / NQ, RR = R + ORDER - 1, NROW = ORDER * RR;
  constexpr int NT = kInterpThreads;
  static_assert(interp_lds_bytes<P, G, ORDER>() <= kMaxLds, "interpolation tile does not fit in LDS");
  static_assert(K1 <= NT, "twiddle table load assumes K1 <= workgroup size");
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + NROW * PC;
  int* nb = reinterpret_cast<int*>(tw + K1);  // head count, body count, overflow count
  TRACE(3, 0);
  const int tid = threadIdx.x;
  if (blockIdx.x == K3 * NQ) {
    if (a.reduce_ev) reduce_ev(a);
    return;
  }
  if (a.N == 0) return;
  static_assert((K3 * NQ) % kXcds == 0, "interpolation tiles do not split over the XCDs");
  const int tile_id = xcd_local(blockIdx.x, K3 * NQ);
  const int z = tile_id / NQ, qs = tile_id - z * NQ, y0 = qs * R;
  const int cap = a.lay.cap;
  const Rec* rec = reinterpret_cast<const Rec*>(a.ws + a.lay.rec);
  const Rec* orec = reinterpret_cast<const Rec*>(a.ws + a.lay.orec);
  const typename P::spec* spec = reinterpret_cast<const typename P::spec*>(a.ws + a.lay.spec);
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  // the bin's buckets (z, qs, head) and (z, qs, body), with the counts the
  // convolution kept for this pass
  const int b0 = (z * NQ + qs) * 2;
  if (tid < 2)
    nb[tid] = min((int)reinterpret_cast<const unsigned*>(a.ws + a.lay.bcnt2)[b0 + tid], cap);
  else if (tid == 2)
    nb[2] = (int)min(reinterpret_cast<const unsigned*>(a.ws + a.lay.ovf)[1],
                     (unsigned)a.lay.orec_max);
  // spectrum rows (jz, r): plane z-p+1+jz, row y0-p+1+r, all x'
  constexpr int NE = KH * NROW;
#pragma unroll 4
  for (int e = tid; e < NE; e += NT) {
    const int r = e % RR, t2 = e / RR, jz = t2 % ORDER, x = t2 / ORDER;
    int zz = z - ORDER + 1 + jz, yy = y0 - ORDER + 1 + r;
    if (zz < 0) zz += K3;
    if (yy < 0) yy += K2;
    buf[(jz * RR + r) * PC + x] = spec_ld(&spec[((size_t)x * K3 + zz) * K2 + yy]);
  }
  if (tid < K1) tw[tid] = twg[tid];
  __syncthreads();
  TRACE(3, 1);
  const int n0 = nb[0], total = n0 + nb[1], novf = nb[2];
  if (total == 0 && novf == 0) return;
  // the first record loads are issued before the transforms
  Rec r;
  if (tid < total) r = rec[tid < n0 ? (size_t)b0 * cap + tid : (size_t)(b0 + 1) * cap + (tid - n0)];
  constexpr int TM = fft_lanes(M);
  if constexpr (x_inv_reg<P, G, ORDER>()) {
    for (int task = tid; task < NROW * TM; task += NT) {
      const int row = task / TM, l = task - row * TM;
      c2r_row_reg<T, K1>(buf + row * PC, l, buf + row * PC, tw);  // the row is its scratch
    }
  } else {
    for (int task = tid; task < NROW * TM; task += NT) {
      const int row = task / TM, l = task - row * TM;
      c2r_pre<T, K1>(buf + row * PC, l, tw);
      fft_pencil<T, M, 1>(buf + row * PC, 1, l, tw, 2);
    }
  }
  __syncthreads();
  TRACE(3, 2);
  auto gather = [&](const Rec& rr) {
    const int gx = rr.g & 1023, gy = (rr.g >> 10) & 1023;
    int xs[ORDER];
#pragma unroll
    for (int jx = 0; jx < ORDER; ++jx) {
      const int x = gx - ORDER + 1 + jx;
      xs[jx] = x < 0 ? x + K1 : x;
    }
    const int ry = gy - y0;
    interpolate<P, ORDER>(
        a, rr,
        [&](int jz, int jy) { return reinterpret_cast<const T*>(buf + (jz * RR + ry + jy) * PC); },
        xs);
  };
  for (int t = tid; t < total; t += NT) {
    Rec rn;
    const int tn = t + NT;
    if (tn < total) rn = rec[tn < n0 ? (size_t)b0 * cap + tn : (size_t)(b0 + 1) * cap + (tn - n0)];
    gather(r);
    r = rn;
  }
  // atoms of full buckets: those of the overflow list that belong to this bin
  for (int o = tid; o < novf; o += NT) {
    const Rec ro = orec[o];
    const int gy = (ro.g >> 10) & 1023, gz = (ro.g >> 20) & 1023;
    if (gz == z && gy / R == qs) gather(ro);
  }
  TRACE(3, 15);
}

// ---------------------------------------------------------------------------
// k_interp_phi: force interpolation from the potential rows in the
// workspace, one (z-plane, y-slice) bin per workgroup, one atom per thread,
// after one k_inv_x launch.  The fused k_interp redoes the inverse x
// transform of p planes and R + p - 1 rows per bin, p (R + p - 1) / R times
// the grid; where that is largest (p >= 6 on K2 K3 >= 16384: 6.8x at 128^3)
// transforming once and gathering from the workspace is faster (measured at
// 128^3: 42 -> 39 us for p = 6; at p = 4 the fused kernel stays ahead, 24
// against 31 us).  A potential row holds a (p-1)-point wrap halo in front,
// so the p x-points of an atom with base index g_x are the consecutive
// entries g_x .. g_x + p - 1.
// ---------------------------------------------------------------------------
template <class P, class G, int ORDER, bool BATCH>
__global__ __launch_bounds__(kInterpThreads) void k_interp_phi(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  using Rec = typename P::rec;
  constexpr int K2 = G::K2, K3 = G::K3;
  constexpr int NQ = nq_of(K2, P::fixed), R = K2 / NQ;
  constexpr int PP = phi_pitch_of(G::K1, ORDER);
  constexpr int NT = kInterpThreads;
  __shared__ int nb[4];  // head count, body count, overflow count
  const int tid = threadIdx.x;
  if (blockIdx.x == K3 * NQ) {
    if (a.reduce_ev) reduce_ev(a);
    return;
  }
  if (a.N == 0) return;
  static_assert((K3 * NQ) % kXcds == 0, "interpolation tiles do not split over the XCDs");
  const int tile_id = xcd_local(blockIdx.x, K3 * NQ);
  const int z = tile_id / NQ, qs = tile_id - z * NQ;
  const int cap = a.lay.cap;
  const Rec* rec = reinterpret_cast<const Rec*>(a.ws + a.lay.rec);
  const Rec* orec = reinterpret_cast<const Rec*>(a.ws + a.lay.orec);
  const T* phi = reinterpret_cast<const T*>(a.ws + a.lay.phi);
  const int b0 = (z * NQ + qs) * 2;
  if (tid < 2)
    nb[tid] = min((int)reinterpret_cast<const unsigned*>(a.ws + a.lay.bcnt2)[b0 + tid], cap);
  else if (tid == 2)
    nb[2] = (int)min(reinterpret_cast<const unsigned*>(a.ws + a.lay.ovf)[1],
                     (unsigned)a.lay.orec_max);
  __syncthreads();
  const int n0 = nb[0], total = n0 + nb[1], novf = nb[2];
  // potential rows (jz, jy) of an atom: plane z-p+1+jz, row g_y-p+1+jy
  int zrow[ORDER];
#pragma unroll
  for (int jz = 0; jz < ORDER; ++jz) {
    int zz = z - ORDER + 1 + jz;
    if (zz < 0) zz += K3;
    zrow[jz] = zz * K2;
  }
  auto gather = [&](const Rec& rr) {
    const int gx = rr.g & 1023, gy = (rr.g >> 10) & 1023;
    int xs[ORDER];
#pragma unroll
    for (int jx = 0; jx < ORDER; ++jx) xs[jx] = gx + jx;
    interpolate<P, ORDER>(
        a, rr,
        [&](int jz, int jy) {
          int yy = gy - ORDER + 1 + jy;
          if (yy < 0) yy += K2;
          return phi + (size_t)(zrow[jz] + yy) * PP;
        },
        xs);
  };
  for (int t = tid; t < total; t += NT)
    gather(rec[t < n0 ? (size_t)b0 * cap + t : (size_t)(b0 + 1) * cap + (t - n0)]);
  // atoms of full buckets: those of the overflow list that belong to this bin
  for (int o = tid; o < novf; o += NT) {
    const Rec ro = orec[o];
    const int gy = (ro.g >> 10) & 1023, gz = (ro.g >> 20) & 1023;
    if (gz == z && gy / R == qs) gather(ro);
  }
}

// ---------------------------------------------------------------------------
// Host-side dispatch over (precision, grid shape, order).
// ---------------------------------------------------------------------------
template <int V>
using ic = std::integral_constant<int, V>;

// Launch with optional timing events attached to the dispatch itself (the
// kernel's own start and end), or plainly.  Batched launches add a second
// grid dimension over the systems of the batch.
template <typename Kern>
hipError_t launch(Kern kernel, dim3 grid, dim3 block, size_t lds, hipStream_t s, const Timing& t,
                  const Args& a, const BatchArgs* bt) {
  static const BatchArgs kNoBatch{};
  const BatchArgs& b = bt != nullptr ? *bt : kNoBatch;
  if (bt != nullptr) grid.y = bt->n;
  if (t.start != nullptr || t.stop != nullptr)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, t.start, t.stop, 0u, a, b);
  else
    kernel<<<grid, block, lds, s>>>(a, b);
  return hipGetLastError();
}

// A launch that is skipped still closes its timing window.
static inline hipError_t skip(hipStream_t s, const Timing& t) {
  if (t.start == nullptr) return hipSuccess;
  hipError_t e = hipEventRecord(t.start, s);
  return e == hipSuccess ? hipEventRecord(t.stop, s) : e;
}

// Supported grids: cubic K = 16, 24, 32, 36, 48, 64, 72, 96, 128, and the
// non-cubic shapes 32 x 32 x 64, 64 x 64 x 128 and 48 x 32 x 64 (x, y, z).
template <class F>
hipError_t with_grid(int K1, int K2, int K3, F&& f) {
  if (K1 == K2 && K2 == K3) {
    switch (K1) {
      case 16: return f(Grid<16, 16, 16>{});
      case 24: return f(Grid<24, 24, 24>{});
      case 32: return f(Grid<32, 32, 32>{});
      case 36: return f(Grid<36, 36, 36>{});
      case 48: return f(Grid<48, 48, 48>{});
      case 64: return f(Grid<64, 64, 64>{});
      case 72: return f(Grid<72, 72, 72>{});
      case 96: return f(Grid<96, 96, 96>{});
      case 128: return f(Grid<128, 128, 128>{});
      default: return hipErrorInvalidValue;
    }
  }
  if (K1 == 32 && K2 == 32 && K3 == 64) return f(Grid<32, 32, 64>{});
  if (K1 == 64 && K2 == 64 && K3 == 128) return f(Grid<64, 64, 128>{});
  if (K1 == 48 && K2 == 32 && K3 == 64) return f(Grid<48, 32, 64>{});
  return hipErrorInvalidValue;
}
template <class F>
hipError_t with_order(int p, F&& f) {
  switch (p) {
    case 4: return f(ic<4>{});
    case 6: return f(ic<6>{});
    default: return hipErrorInvalidValue;
  }
}

template <class F>
hipError_t with_batch(const BatchArgs* bt, F&& f) {
  if (bt != nullptr) return f(std::true_type{});
  return f(std::false_type{});
}

// Which variants of the convolution and interpolation a (precision, grid,
// order) combination can run: the fused column must fit in LDS, the split
// passes need whole chunks of rows per workgroup, the fused interpolation
// tile must fit in LDS.
template <class P, class G>
__host__ __device__ constexpr bool conv_fused_ok() {
  return conv_lds_bytes<P, G>() <= kMaxLds;
}
template <class P, class G>
__host__ __device__ constexpr bool conv_split_ok() {
  return pass_cz<G>() >= 1 && G::K3 % pass_cz<G>() == 0 &&
         pass_cz<G>() * fft_lanes(G::K2) == kPassThreads && pass_cy<G>() >= 1 &&
         G::K2 % pass_cy<G>() == 0 && pass_cy<G>() * fft_lanes(G::K3) == kPassThreads &&
         conv_y_lds_bytes<P, G>() <= kMaxLds && conv_z_lds_bytes<P, G>() <= kMaxLds;
}
template <class P, class G>
__host__ __device__ constexpr bool conv_reg_ok() {
  return conv_reg_shape<G>() && conv_reg_lds_bytes<P, G>() <= kMaxLds;
}
template <class P, class G, int ORDER>
__host__ __device__ constexpr bool interp_fused_ok() {
  return interp_lds_bytes<P, G, ORDER>() <= kMaxLds;
}

template <class P, class G, int O, bool B>
hipError_t raise_all_lds_limits() {
  const hipFuncAttribute attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipFuncSetAttribute((const void*)k_spread_x<P, G, O, B>, attr,
                                     (int)spread_lds_bytes<P, G>());
  if constexpr (conv_split_ok<P, G>()) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_conv_y<P, G, -1, B>, attr,
                              (int)conv_y_lds_bytes<P, G>());
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_conv_y<P, G, 1, B>, attr,
                              (int)conv_y_lds_bytes<P, G>());
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_conv_z<P, G, B>, attr, (int)conv_z_lds_bytes<P, G>());
  }
  if constexpr (conv_fused_ok<P, G>()) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_conv<P, G, B>, attr, (int)conv_lds_bytes<P, G>());
  }
  if constexpr (conv_reg_ok<P, G>()) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_conv_reg<P, G, B>, attr,
                              (int)conv_reg_lds_bytes<P, G>());
  }
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_inv_x<P, G, O, B>, attr, (int)inv_x_lds_bytes<P, G, O>());
  if constexpr (interp_fused_ok<P, G, O>()) {
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_interp<P, G, O, B>, attr,
                              (int)interp_lds_bytes<P, G, O>());
  }
  return e;
}

template <class P>
hipError_t prepare_p(int K1, int K2, int K3, int order) {
  return with_grid(K1, K2, K3, [&](auto gc) {
    using G = decltype(gc);
    return with_order(order, [&](auto oc) {
      constexpr int O = decltype(oc)::value;
      hipError_t e = raise_all_lds_limits<P, G, O, false>();
      return e == hipSuccess ? raise_all_lds_limits<P, G, O, true>() : e;
    });
  });
}

template <class P>
unsigned variants_p(int K1, int K2, int K3, int order) {
  unsigned v = 0;
  (void)with_grid(K1, K2, K3, [&](auto gc) {
    using G = decltype(gc);
    return with_order(order, [&](auto oc) {
      constexpr int O = decltype(oc)::value;
      v = (conv_fused_ok<P, G>() ? kVarConvFused : 0u) | (conv_split_ok<P, G>() ? kVarConvSplit : 0u) |
          (conv_reg_ok<P, G>() ? kVarConvReg : 0u) |
          (interp_fused_ok<P, G, O>() ? kVarInterpFused : 0u) | kVarInterpSplit;
      return hipSuccess;
    });
  });
  return v;
}

template <class P>
hipError_t launch_bin_p(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  if (a.n_chunks == 0) return skip(s, t);
  return with_batch(bt, [&](auto bc) {
    constexpr bool B = decltype(bc)::value;
    return launch(k_bin<P, B>, dim3(a.n_chunks), dim3(a.bin_chunk), 0, s, t, a, bt);
  });
}

template <class P>
hipError_t launch_spread_x_p(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_grid(a.K1, a.K2, a.K3, [&](auto gc) {
    using G = decltype(gc);
    return with_order(a.order, [&](auto oc) {
      constexpr int O = decltype(oc)::value;
      return with_batch(bt, [&](auto bc) {
        constexpr bool B = decltype(bc)::value;
        return launch(k_spread_x<P, G, O, B>, dim3(G::K3 * nq_of(G::K2, P::fixed)),
                      dim3(spread_threads<B>()), spread_lds_bytes<P, G>(), s, t, a, bt);
      });
    });
  });
}

template <class P>
hipError_t launch_conv_p(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_grid(a.K1, a.K2, a.K3, [&](auto gc) {
    using G = decltype(gc);
    return with_batch(bt, [&](auto bc) {
      constexpr bool B = decltype(bc)::value;
      constexpr int KH = G::K1 / 2 + 1;
      if (a.conv_mode == kConvSplit) {
        if constexpr (conv_split_ok<P, G>()) {
          // three launches; the timing window spans all of them
          const Timing first{t.start, nullptr}, last{nullptr, t.stop};
          const dim3 ygrid(KH * (G::K3 / pass_cz<G>()));
          hipError_t e = launch(k_conv_y<P, G, -1, B>, ygrid, dim3(kPassThreads),
                                conv_y_lds_bytes<P, G>(), s, first, a, bt);
          if (e == hipSuccess)  // column chunks and the counts/headroom workgroup
            e = launch(k_conv_z<P, G, B>, dim3(KH * (G::K2 / pass_cy<G>()) + 1),
                       dim3(kPassThreads), conv_z_lds_bytes<P, G>(), s, Timing(), a, bt);
          if (e == hipSuccess)
            e = launch(k_conv_y<P, G, 1, B>, ygrid, dim3(kPassThreads), conv_y_lds_bytes<P, G>(),
                       s, last, a, bt);
          return e;
        }
      } else if (a.conv_mode == kConvFused) {
        if constexpr (conv_fused_ok<P, G>()) {
          const int blocks = KH + 1;  // columns and the counts/headroom workgroup
          return launch(k_conv<P, G, B>, dim3(blocks), dim3(conv_block<P, G, B>()),
                        conv_lds_bytes<P, G>(), s, t, a, bt);
        }
      } else if (a.conv_mode == kConvReg) {
        if constexpr (conv_reg_ok<P, G>()) {
          return launch(k_conv_reg<P, G, B>, dim3(KH + 1), dim3(conv_reg_threads<G>()),
                        conv_reg_lds_bytes<P, G>(), s, t, a, bt);
        }
      }
      return hipErrorInvalidValue;
    });
  });
}

template <class P>
hipError_t launch_inv_x_p(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_grid(a.K1, a.K2, a.K3, [&](auto gc) {
    using G = decltype(gc);
    return with_order(a.order, [&](auto oc) {
      constexpr int O = decltype(oc)::value;
      return with_batch(bt, [&](auto bc) {
        constexpr bool B = decltype(bc)::value;
        return launch(k_inv_x<P, G, O, B>, dim3(G::K3), dim3(kPlaneThreads),
                      inv_x_lds_bytes<P, G, O>(), s, t, a, bt);
      });
    });
  });
}

template <class P>
hipError_t launch_interp_p(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_grid(a.K1, a.K2, a.K3, [&](auto gc) {
    using G = decltype(gc);
    return with_order(a.order, [&](auto oc) {
      constexpr int O = decltype(oc)::value;
      return with_batch(bt, [&](auto bc) {
        constexpr bool B = decltype(bc)::value;
        const int blocks = G::K3 * nq_of(G::K2, P::fixed) + ((a.reduce_ev || B) ? 1 : 0);
        if (a.interp_mode == kInterpSplit) {
          // inverse x transform once per plane, then the gather; the timing
          // window spans both launches
          const Timing first{t.start, nullptr}, last{nullptr, t.stop};
          hipError_t e = launch(k_inv_x<P, G, O, B>, dim3(G::K3), dim3(kPlaneThreads),
                                inv_x_lds_bytes<P, G, O>(), s, first, a, bt);
          if (e == hipSuccess)
            e = launch(k_interp_phi<P, G, O, B>, dim3(blocks), dim3(kInterpThreads), 0, s, last,
                       a, bt);
          return e;
        }
        if constexpr (interp_fused_ok<P, G, O>()) {
          if (a.interp_mode == kInterpFused)
            return launch(k_interp<P, G, O, B>, dim3(blocks), dim3(kInterpThreads),
                          interp_lds_bytes<P, G, O>(), s, t, a, bt);
        }
        return hipErrorInvalidValue;
      });
    });
  });
}

// The launch table of one precision (each precision's kernels are compiled
// in a translation unit of their own).
template <class P>
PrecOps make_ops() {
  PrecOps o;
  o.prepare = &prepare_p<P>;
  o.variants = &variants_p<P>;
  o.bin = &launch_bin_p<P>;
  o.spread_x = &launch_spread_x_p<P>;
  o.conv = &launch_conv_p<P>;
  o.inv_x = &launch_inv_x_p<P>;
  o.interp = &launch_interp_p<P>;
#ifdef SPME_TRACE
  o.trace_set = &trace_set_here;
#endif
  return o;
}
}  // namespace spme
