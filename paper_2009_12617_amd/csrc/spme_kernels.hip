// HIP kernels of the SPME reciprocal-space step for gfx950 (CDNA4).
//
// One step is six launches on one stream:
//   k_bin       fractional coordinates, base grid index and offsets of each
//               atom; a per-chunk counting sort of the atoms by (base z,
//               y slice) -- the GPU counterpart of the
//               paper's atom reordering for hazard suppression (§III.A.1, §V.C)
//   k_spread_x  one y slice of one z-plane per workgroup: every atom whose
//               support covers the slice adds its contributions into an LDS
//               tile in 64-bit fixed point (integer adds commute, so the grid
//               is bit-identical whatever the order); the finished rows are
//               converted to FP32 and transformed along x (real-to-complex)
//   k_fft_y     one z-plane per workgroup: y transforms (§III.A.2: "each
//               slab runs independently to compute X and Y transforms")
//   k_pencil    one y row (or half of it) per workgroup: z transforms,
//               multiplication by the influence function with FP64 energy and
//               virial partials, inverse z transforms (§III.A.2: "Z direction
//               transforms, multiply by Green's function data, compute Z^-1
//               transforms")
//   k_inv_xy    one z-plane per workgroup: inverse y and complex-to-real x
//               transforms; potential rows written with a (p-1)-point wrap
//               halo so interpolation reads contiguous runs; one extra
//               workgroup adds the energy/virial partial rows
//   k_gather    one atom per thread: B-spline weights and derivatives, p^3
//               potential reads, forces scattered back to the caller's atom
//               order (§III.A.3)
// The paper's two all-to-all corner turns become the HBM round trips between
// plane and pencil passes.
#include <hip/hip_ext.h>

#include <type_traits>

#include "spme_device.h"
#include "spme_internal.h"
#include "../../include/spme.h"

namespace spme {

// Optional phase trace (build with -DSPME_TRACE): thread 0 of each workgroup
// stamps the 100 MHz wall clock at phase boundaries into
// trace[kernel][workgroup][phase]; kernels 0..5 in launch order, phase 0 at
// entry and 15 at exit.
#ifdef SPME_TRACE
__device__ unsigned long long* g_trace;
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

struct PFixed {
  using real = float;
  using acc = unsigned long long;
  using rec = RecF;
  static constexpr bool fixed = true;
};
struct PDouble {
  using real = double;
  using acc = double;
  using rec = RecD;
  static constexpr bool fixed = false;
};

// Row pitch of an LDS grid tile in 8-byte units.  Fixed point: K int64
// values per row (the half spectrum of K/2+1 float2 fits in place).  FP64:
// room for K/2+1 double2.  The extra unit skews rows across LDS banks.
template <class P>
__host__ __device__ constexpr int tile_pitch(int K) { return P::fixed ? K + 1 : K + 4; }

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

// Exclusive prefix sum over the block; wsum needs 32 ints.  Every thread
// must call it; the caller synchronises before reusing wsum.
__device__ int block_exclusive_scan(int v, int* wsum, int* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    int w = (lane < nw) ? wsum[lane] : 0;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      const int y = __shfl_up(w, d, 64);
      if (lane >= d) w += y;
    }
    if (lane < nw) wsum[16 + lane] = w;
  }
  __syncthreads();
  *total = wsum[16 + nw - 1];
  return (wave > 0 ? wsum[16 + wave - 1] : 0) + x - v;
}

// Sums of V doubles over the block in a fixed order: every thread stores its
// values, 16 threads per value add consecutive runs of blockDim/16 entries,
// then thread c < V adds the 16 run sums of value c in order and returns it
// (other threads return 0).  red needs block_sum_doubles(V, blockDim)
// doubles; the caller synchronises before reusing red.
__host__ __device__ constexpr int block_sum_doubles(int V, int threads) { return V * (threads + 16); }

template <int V>
__device__ double block_sums(const double* v, double* red) {
  const int n = blockDim.x, tid = threadIdx.x;
#pragma unroll
  for (int c = 0; c < V; ++c) red[c * n + tid] = v[c];
  __syncthreads();
  double* part = red + V * n;
  const int run = n / 16;
  if (tid < V * 16) {
    const int c = tid / 16, k = tid - c * 16;
    const double* src = red + c * n + k * run;
    double s = 0.0;
    for (int i = 0; i < run; ++i) s += src[i];
    part[tid] = s;
  }
  __syncthreads();
  double s = 0.0;
  if (tid < V) {
#pragma unroll
    for (int k = 0; k < 16; ++k) s += part[tid * 16 + k];
  }
  return s;
}

// ---------------------------------------------------------------------------
// k_bin: one chunk of kChunk atoms per workgroup.
// ---------------------------------------------------------------------------
template <class P, bool BATCH>
__global__ __launch_bounds__(kBinThreads) void k_bin(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  if (BATCH && (int)blockIdx.x >= a.n_chunks) return;
  using Rec = typename P::rec;
  using T = typename P::real;
  __shared__ int hist[kMaxBins];
  __shared__ int wsum[32];
  __shared__ double red[block_sum_doubles(1, kBinThreads)];
  TRACE(0, 0);
  const int K = a.K, nq = nq_of(a.K), rows = K / nq, nbins = 2 * K * nq;
  const int c = blockIdx.x, tid = threadIdx.x;
  int2* cnt = reinterpret_cast<int2*>(a.ws + a.lay.cnt) + (size_t)c * nbins;
  Rec* rec = reinterpret_cast<Rec*>(a.ws + a.lay.rec) + (size_t)c * kChunk;
  unsigned* flags = reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl);
  for (int b = tid; b < nbins; b += kBinThreads) hist[b] = 0;
  __syncthreads();
  TRACE(0, 1);

  // one atom per thread
  const int i = c * kChunk + tid;
  Rec r;
  int bin = -1, rank = 0;
  double v[1] = {0.0};
  if (i < a.N) {
    int g[3];
    double w[3];
    bool ok = true;
#pragma unroll
    for (int d = 0; d < 3; ++d) ok &= grid_coord(a.pos[3 * (size_t)i + d], a.invL[d], K, &g[d], &w[d]);
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
    r.idx = i;
    // bin (z, y slice, head/body): the head holds the atoms whose support
    // also reaches the slice below (g_y mod rows < p - 1)
    const int sl = g[1] / rows;
    bin = (g[2] * nq + sl) * 2 + ((g[1] - sl * rows) >= a.order - 1 ? 1 : 0);
    rank = atomicAdd(&hist[bin], 1);
  }
  // sum |q| of the chunk (fixed-point headroom), before any global store so
  // that the barriers below do not wait on outstanding writes
  const double qsum = block_sums<1>(v, red);
  TRACE(0, 2);
  // exclusive scan of the bin counts, one bin per thread
  const int h = (tid < nbins) ? hist[tid] : 0;
  int total;
  const int ex = block_exclusive_scan(h, wsum, &total);
  if (tid < nbins) hist[tid] = ex;  // own slot: read above by this thread only
  __syncthreads();
  TRACE(0, 3);
  if (bin >= 0) rec[hist[bin] + rank] = r;
  if (tid < nbins) cnt[tid] = make_int2(h, ex);
  if (tid == 0) reinterpret_cast<double*>(a.ws + a.lay.absq)[c] = qsum;
  TRACE(0, 15);
}

// ---------------------------------------------------------------------------
// k_spread_x: charge spreading of one y slice of one z-plane, then the x
// real-to-complex FFT of its rows.
// ---------------------------------------------------------------------------
template <class P, int K>
__host__ __device__ constexpr size_t spread_lds_bytes() {
  return (size_t)(K / nq_of(K)) * tile_pitch<P>(K) * 8 +
         (size_t)K * sizeof(cplx<typename P::real>) +
         (size_t)(2 * kSegPerThread * kSpreadThreads + 2 + 32) * sizeof(int) +
         kItemMap * sizeof(unsigned short);
}

template <class P, int K, int ORDER, bool BATCH>
__global__ __launch_bounds__(kSpreadThreads) void k_spread_x(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  using Acc = typename P::acc;
  using Rec = typename P::rec;
  constexpr int M = K / 2, KH = K / 2 + 1;
  constexpr int NQ = nq_of(K), R = K / NQ;
  constexpr int PITCH = tile_pitch<P>(K);
  extern __shared__ __align__(16) unsigned char smem[];
  Acc* tile = reinterpret_cast<Acc*>(smem);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + (size_t)R * PITCH * 8);
  int* segpre = reinterpret_cast<int*>(tw + K);
  int* segbeg = segpre + kSegPerThread * kSpreadThreads + 2;
  int* wsum = segbeg + kSegPerThread * kSpreadThreads;
  unsigned short* imap = reinterpret_cast<unsigned short*>(wsum + 32);

  TRACE(1, 0);
  static_assert((K * NQ) % kXcds == 0, "spreading tiles do not split over the XCDs");
  const int tile_id = xcd_local(blockIdx.x, K * NQ);
  const int z = tile_id / NQ, qs = tile_id - z * NQ, y0 = qs * R;
  const int tid = threadIdx.x;
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < K; i += kSpreadThreads) tw[i] = twg[i];
  for (int i = tid; i < R * PITCH; i += kSpreadThreads) tile[i] = Acc(0);
  const int2* cnt = reinterpret_cast<const int2*>(a.ws + a.lay.cnt);
  const Rec* rec = reinterpret_cast<const Rec*>(a.ws + a.lay.rec);
  const double scale = ldexp(1.0, a.frac_bits);
  __syncthreads();
  TRACE(1, 1);

  // --- spreading.  The tile (rows y0 .. y0+R-1 of plane z) receives the
  // atoms whose base z index b lies in z .. z+p-1 (mod K) -- for b = z + j
  // the plane is support point jz = p-1-j -- and whose base y index lies in
  // this slice, or in the head (first p-1 rows) of the next slice: an atom
  // touches rows g_y-p+1 .. g_y.  A segment is the run of one such bin
  // (z, slice, head/body) inside one sorted chunk; segments are taken
  // kSpreadThreads at a time and their items are numbered consecutively.  An
  // LDS map gives each item's segment; each thread then owns kItems items per
  // pass so that their record loads overlap.
  constexpr int kItems = 4;
  constexpr int NB = 2 * K * NQ;
  constexpr int SPJ = 3;  // segments per (chunk, j): own head, own body, next head
  constexpr int SPT = kSegPerThread;
  const int nseg = a.n_chunks * ORDER * SPJ;
  for (int s0 = 0; s0 < nseg; s0 += SPT * kSpreadThreads) {
    const int ns = min(SPT * kSpreadThreads, nseg - s0);
    // each thread describes SPT consecutive segments
    int len[SPT], beg[SPT], mine = 0;
#pragma unroll
    for (int k = 0; k < SPT; ++k) {
      const int sl = tid * SPT + k;
      len[k] = 0;
      beg[k] = 0;
      if (sl < ns) {
        const int seg = s0 + sl;
        const int c = seg / (SPJ * ORDER), rem = seg - c * SPJ * ORDER;
        const int j = rem / SPJ, d = rem - j * SPJ;
        int bz = z + j;
        if (bz >= K) bz -= K;
        int by = qs + (d == 2 ? 1 : 0);
        if (by >= NQ) by -= NQ;
        const int2 v = cnt[(size_t)c * NB + (bz * NQ + by) * 2 + (d == 1 ? 1 : 0)];
        len[k] = v.x;
        beg[k] = c * kChunk + v.y;
      }
      mine += len[k];
    }
    int total;
    const int ex = block_exclusive_scan(mine, wsum, &total);
    int pre[SPT];
    {
      int run = ex;
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        const int sl = tid * SPT + k;
        pre[k] = run;
        if (sl < ns) {
          segpre[sl] = run;
          segbeg[sl] = beg[k];
        }
        run += len[k];
      }
    }
    if (tid == 0) segpre[ns] = total;
    TRACE(1, 4);
    for (int w0 = 0; w0 < total; w0 += kItemMap) {
      const int wn = min(kItemMap, total - w0);
      // map the items of this window to their segments
#pragma unroll
      for (int k = 0; k < SPT; ++k) {
        const int lo = max(pre[k], w0), hi = min(pre[k] + len[k], w0 + wn);
        for (int t = lo; t < hi; ++t) imap[t - w0] = (unsigned short)(tid * SPT + k);
      }
      __syncthreads();
      TRACE(1, 5);
      for (int it = 0; it < wn; it += kItems * kSpreadThreads) {
        int idx[kItems], jz[kItems];
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
          const int t = it + u * kSpreadThreads + tid;
          jz[u] = -1;
          idx[u] = 0;
          if (t < wn) {
            const int sg = imap[t];
            idx[u] = segbeg[sg] + (w0 + t - segpre[sg]);
            jz[u] = ORDER - 1 - ((s0 + sg) % (SPJ * ORDER)) / SPJ;
          }
        }
        Rec r[kItems];
#pragma unroll
        for (int u = 0; u < kItems; ++u)
          if (jz[u] >= 0) r[u] = rec[idx[u]];
#pragma unroll
        for (int u = 0; u < kItems; ++u) {
          if (jz[u] < 0) continue;
          const int gx = r[u].g & 1023, gy = (r[u].g >> 10) & 1023;
          T tx[ORDER], ty[ORDER], tz[ORDER];
          bspline<ORDER>(r[u].w[0], tx, (T*)nullptr);
          bspline<ORDER>(r[u].w[1], ty, (T*)nullptr);
          bspline<ORDER>(r[u].w[2], tz, (T*)nullptr);
          int xs[ORDER];
#pragma unroll
          for (int jx = 0; jx < ORDER; ++jx) {
            const int x = gx - ORDER + 1 + jx;
            xs[jx] = x < 0 ? x + K : x;
          }
          if constexpr (P::fixed) {
#pragma clang fp contract(off)
            const float cz = r[u].q * pick<ORDER>(tz, jz[u]);  // product order z, y, x
#pragma unroll
            for (int jy = 0; jy < ORDER; ++jy) {
              int dy = gy - ORDER + 1 + jy - y0;
              if (dy < 0) dy += K;
              if (dy >= R) continue;
              Acc* row = tile + dy * PITCH;
              const float cy = cz * ty[jy];
#pragma unroll
              for (int jx = 0; jx < ORDER; ++jx)
                atomicAdd(&row[xs[jx]], (unsigned long long)to_fixed(cy * tx[jx], scale));
            }
          } else {
            const double cz = r[u].q * pick<ORDER>(tz, jz[u]);
#pragma unroll
            for (int jy = 0; jy < ORDER; ++jy) {
              int dy = gy - ORDER + 1 + jy - y0;
              if (dy < 0) dy += K;
              if (dy >= R) continue;
              Acc* row = tile + dy * PITCH;
              const double cy = cz * ty[jy];
#pragma unroll
              for (int jx = 0; jx < ORDER; ++jx) atomicAdd(&row[xs[jx]], cy * tx[jx]);
            }
          }
        }
      }
      __syncthreads();
    }
  }
  TRACE(1, 2);

  if (a.keep_grid) {
    Acc* dbg = reinterpret_cast<Acc*>(a.ws + a.lay.dbg) + ((size_t)z * K + y0) * K;
    for (int i = tid; i < R * K; i += kSpreadThreads) dbg[i] = tile[(i / K) * PITCH + (i % K)];
    __syncthreads();  // the x transform below overwrites the tile in place
  }

  // --- x: real-to-complex, one row per group of fft_lanes(M) lanes.
  constexpr int TM = fft_lanes(M);
  for (int task = tid; task < R * TM; task += kSpreadThreads) {
    const int y = task / TM, l = task - y * TM;
    cplx<T>* row = reinterpret_cast<cplx<T>*>(tile + y * PITCH);
    if constexpr (P::fixed) {
      // int64 -> float in place: x_j at float slot j, so the row reads as the
      // packed complex sequence z_n = x_{2n} + i x_{2n+1}
      const double inv_scale = ldexp(1.0, -a.frac_bits);
      constexpr int PER = K / TM;
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
    r2c_post<T, K>(row, l, tw);
  }
  __syncthreads();
  TRACE(1, 3);

  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.ws + a.lay.spec) + ((size_t)z * K + y0) * KH;
  constexpr int PC = P::fixed ? PITCH : PITCH / 2;
  const cplx<T>* tc = reinterpret_cast<const cplx<T>*>(tile);
  for (int i = tid; i < R * KH; i += kSpreadThreads) {
    const int y = i / KH, x = i - y * KH;
    spec[i] = tc[y * PC + x];
  }
  TRACE(1, 15);
}

// ---------------------------------------------------------------------------
// k_fft_y: forward y FFT of one z-plane of the half spectrum.
// ---------------------------------------------------------------------------
template <class P, int K>
__host__ __device__ constexpr size_t plane_lds_bytes() {
  return (size_t)K * (K / 2 + 2) * sizeof(cplx<typename P::real>) +
         (size_t)K * sizeof(cplx<typename P::real>);
}
// k_fft_y also hosts the fixed-point headroom workgroup.
template <class P, int K>
__host__ __device__ constexpr size_t fft_y_lds_bytes() {
  return plane_lds_bytes<P, K>() > block_sum_doubles(1, kPlaneThreads) * sizeof(double)
             ? plane_lds_bytes<P, K>()
             : block_sum_doubles(1, kPlaneThreads) * sizeof(double);
}
// k_inv_xy also hosts the energy/virial reduction workgroup.
template <class P, int K>
__host__ __device__ constexpr size_t inv_lds_bytes() {
  return plane_lds_bytes<P, K>() > block_sum_doubles(7, kPlaneThreads) * sizeof(double)
             ? plane_lds_bytes<P, K>()
             : block_sum_doubles(7, kPlaneThreads) * sizeof(double);
}

template <class P, int K, bool BATCH>
__global__ __launch_bounds__(kPlaneThreads) void k_fft_y(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  constexpr int KH = K / 2 + 1, PC = KH + 1;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = pl + K * PC;
  TRACE(2, 0);
  const int tid = threadIdx.x;
  if (blockIdx.x == K) {
    // the extra workgroup (fixed point only): sum |q| 2^F must stay below
    // 2^51 so that every contribution and grid value is exact in FP64 and the
    // rounding of to_fixed holds
    const double* absq = reinterpret_cast<const double*>(a.ws + a.lay.absq);
    double v[1] = {0.0};
    for (int c = tid; c < a.n_chunks; c += kPlaneThreads) v[0] += absq[c];
    const double qsum = block_sums<1>(v, reinterpret_cast<double*>(smem));
    if (tid == 0 && qsum * ldexp(1.0, a.frac_bits) >= 2251799813685248.0)
      atomicOr(reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl), PME_FLAG_OVERFLOW);
    return;
  }
  static_assert(K % kXcds == 0, "planes do not split over the XCDs");
  const int z = xcd_local(blockIdx.x, K);
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.ws + a.lay.spec) + (size_t)z * K * KH;
  for (int i = tid; i < K * KH; i += kPlaneThreads) {
    const int y = i / KH, x = i - y * KH;
    pl[y * PC + x] = spec[i];
  }
  for (int i = tid; i < K; i += kPlaneThreads) tw[i] = twg[i];
  __syncthreads();
  TRACE(2, 1);
  constexpr int TK = fft_lanes(K);
  for (int task = tid; task < KH * TK; task += kPlaneThreads) {
    const int x = task / TK, l = task - x * TK;
    fft_pencil<T, K, -1>(pl + x, PC, l, tw, 1);
  }
  __syncthreads();
  TRACE(2, 2);
  for (int i = tid; i < K * KH; i += kPlaneThreads) {
    const int y = i / KH, x = i - y * KH;
    spec[i] = pl[y * PC + x];
  }
  TRACE(2, 15);
}

// ---------------------------------------------------------------------------
// k_pencil: z FFT, influence function with energy/virial, inverse z FFT.
// ---------------------------------------------------------------------------
template <class P, int K>
__host__ __device__ constexpr size_t pencil_lds_bytes() {
  constexpr int KH = K / 2 + 1, XW = (KH + pencil_xsplit(K) - 1) / pencil_xsplit(K);
  return (size_t)K * (XW + 1) * sizeof(cplx<typename P::real>) +
         (size_t)K * sizeof(cplx<typename P::real>) + 3 * (size_t)K * sizeof(double) +
         block_sum_doubles(7, kPencilThreads) * sizeof(double);
}

template <class P, int K, bool BATCH>
__global__ __launch_bounds__(kPencilThreads) void k_pencil(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  constexpr int KH = K / 2 + 1;
  constexpr int XS = pencil_xsplit(K);
  constexpr int XW = (KH + XS - 1) / XS;
  constexpr int PW = XW + 1;
  constexpr double PI = 3.14159265358979323846;
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* buf = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = buf + K * PW;
  double* bs = reinterpret_cast<double*>(tw + K);
  double* red = bs + 3 * K;

  TRACE(3, 0);
  const int tid = threadIdx.x;
  const int y = blockIdx.x / XS;
  const int x0 = (blockIdx.x - y * XS) * XW;
  const int xw = min(XW, KH - x0);
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.ws + a.lay.spec);
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  const double* bsg = reinterpret_cast<const double*>(a.ws + a.lay.bsq);
  for (int i = tid; i < K * XW; i += kPencilThreads) {
    const int zz = i / XW, xx = i - zz * XW;
    if (xx < xw) buf[zz * PW + xx] = spec[((size_t)zz * K + y) * KH + x0 + xx];
  }
  for (int i = tid; i < K; i += kPencilThreads) tw[i] = twg[i];
  {
    // T_a(m) = |b_a(m)|^2 exp(-pi^2 mt^2 / (beta L_a)^2) per axis
    const double fac = PI * PI / (a.beta * a.beta);
    for (int i = tid; i < 3 * K; i += kPencilThreads) {
      const int ax = i / K, m = i - ax * K;
      const int mt = (m <= K / 2) ? m : m - K;
      const double u = mt * a.invL[ax];
      bs[i] = bsg[i] * exp(-fac * u * u);
    }
  }
  __syncthreads();
  TRACE(3, 1);

  constexpr int TK = fft_lanes(K);
  for (int task = tid; task < XW * TK; task += kPencilThreads) {
    const int xx = task / TK, l = task - xx * TK;
    if (xx < xw) fft_pencil<T, K, -1>(buf + xx, PW, l, tw, 1);
  }
  __syncthreads();
  TRACE(3, 2);

  // G(m) = c B(m) exp(-pi^2 |m|^2 / beta^2) / (pi V |m|^2).  In an
  // orthorhombic cell B exp(-pi^2|m|^2/beta^2) = T_x(m1) T_y(m2) T_z(m3).
  // The half spectrum counts every m1 = 1 .. K/2-1 twice (its Hermitian
  // partner), m1 = 0 and m1 = K/2 once.
  const double pref = a.coulomb / (PI * a.volume);
  const double fac = PI * PI / (a.beta * a.beta);
  const int my = (y <= K / 2) ? y : y - K;
  const double mvy = my * a.invL[1];
  const double ny = (2 * y == K) ? 0.0 : mvy;
  const double Ty = bs[K + y];
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int i = tid; i < K * XW; i += kPencilThreads) {
    const int zz = i / XW, xx = i - zz * XW;
    if (xx >= xw) continue;
    const int m1 = x0 + xx;
    const int mz = (zz <= K / 2) ? zz : zz - K;
    const double mvx = m1 * a.invL[0], mvz = mz * a.invL[2];
    // a Nyquist index aliases +K/2 and -K/2 equally: its sign-odd products vanish
    const double nx = (2 * m1 == K) ? 0.0 : mvx, nz = (2 * zz == K) ? 0.0 : mvz;
    const double msq = mvx * mvx + mvy * mvy + mvz * mvz;
    double G = 0.0, t = 0.0;
    if (m1 != 0 || y != 0 || zz != 0) {
      const double inv = 1.0 / msq;
      G = pref * bs[m1] * Ty * bs[2 * K + zz] * inv;
      t = 2.0 * (inv + fac);
    }
    cplx<T> f = buf[zz * PW + xx];
    const double f2 = (double)f.x * (double)f.x + (double)f.y * (double)f.y;
    const double e = ((m1 == 0 || 2 * m1 == K) ? 0.5 : 1.0) * G * f2;
    acc[0] += e;
    acc[1] += e * (1.0 - t * mvx * mvx);
    acc[2] += e * (1.0 - t * mvy * mvy);
    acc[3] += e * (1.0 - t * mvz * mvz);
    acc[4] -= e * t * nx * ny;
    acc[5] -= e * t * nx * nz;
    acc[6] -= e * t * ny * nz;
    const T g = (T)G;
    buf[zz * PW + xx] = {f.x * g, f.y * g};
  }
  // Energy/virial: fixed-order block sums, one partial row per workgroup,
  // added in workgroup order by the next kernel on the stream.  (Done before
  // the final stores: a barrier after global stores waits for them.)
  const double tot = block_sums<7>(acc, red);
  if (tid < 7) reinterpret_cast<double*>(a.ws + a.lay.partial)[blockIdx.x * 8 + tid] = tot;
  TRACE(3, 3);

  for (int task = tid; task < XW * TK; task += kPencilThreads) {
    const int xx = task / TK, l = task - xx * TK;
    if (xx < xw) fft_pencil<T, K, 1>(buf + xx, PW, l, tw, 1);
  }
  __syncthreads();
  TRACE(3, 4);
  for (int i = tid; i < K * XW; i += kPencilThreads) {
    const int zz = i / XW, xx = i - zz * XW;
    if (xx < xw) spec[((size_t)zz * K + y) * KH + x0 + xx] = buf[zz * PW + xx];
  }
  TRACE(3, 15);
}

// Sum of the energy/virial partial rows in row order by one workgroup.
__device__ void reduce_ev(const Args& a, double* red) {
  const double* partial = reinterpret_cast<const double*>(a.ws + a.lay.partial);
  const int rows = a.lay.pencil_blocks;
  double r[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < rows; b += blockDim.x) {
#pragma unroll
    for (int c = 0; c < 7; ++c) r[c] += partial[b * 8 + c];
  }
  const double tot = block_sums<7>(r, red);
  if (threadIdx.x < 7) a.ev[threadIdx.x] = tot;
}

// (same block size as k_inv_xy's reduction workgroup: identical sum order)
__global__ __launch_bounds__(kPlaneThreads) void k_reduce_ev(Args a) {
  __shared__ double red[block_sum_doubles(7, kPlaneThreads)];
  reduce_ev(a, red);
}

// ---------------------------------------------------------------------------
// k_inv_xy: inverse y FFT and complex-to-real x FFT of one z-plane.
// ---------------------------------------------------------------------------
template <class P, int K, int ORDER, bool BATCH>
__global__ __launch_bounds__(kPlaneThreads) void k_inv_xy(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  constexpr int M = K / 2, KH = K / 2 + 1, PC = KH + 1;
  constexpr int PP = phi_pitch_of(K, ORDER);
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = pl + K * PC;
  TRACE(4, 0);
  const int tid = threadIdx.x;
  if (blockIdx.x == K) {
    // the extra workgroup: energy and virial
    if (a.reduce_ev) reduce_ev(a, reinterpret_cast<double*>(smem));
    return;
  }
  const int z = xcd_local(blockIdx.x, K);
  const cplx<T>* spec = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.spec) + (size_t)z * K * KH;
  for (int i = tid; i < K * KH; i += kPlaneThreads) {
    const int y = i / KH, x = i - y * KH;
    pl[y * PC + x] = spec[i];
  }
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < K; i += kPlaneThreads) tw[i] = twg[i];
  __syncthreads();
  TRACE(4, 1);

  constexpr int TK = fft_lanes(K);
  for (int task = tid; task < KH * TK; task += kPlaneThreads) {
    const int x = task / TK, l = task - x * TK;
    fft_pencil<T, K, 1>(pl + x, PC, l, tw, 1);
  }
  __syncthreads();
  TRACE(4, 2);

  constexpr int TM = fft_lanes(M);
  for (int task = tid; task < K * TM; task += kPlaneThreads) {
    const int y = task / TM, l = task - y * TM;
    cplx<T>* row = pl + y * PC;
    c2r_pre<T, K>(row, l, tw);
    fft_pencil<T, M, 1>(row, 1, l, tw, 2);
  }
  __syncthreads();
  TRACE(4, 3);

  T* phi = reinterpret_cast<T*>(a.ws + a.lay.phi) + (size_t)z * K * PP;
  for (int i = tid; i < K * PP; i += kPlaneThreads) {
    const int y = i / PP, xh = i - y * PP;
    int x = xh - (ORDER - 1);
    if (x < 0) x += K;
    if (x >= K) x -= K;
    phi[i] = reinterpret_cast<const T*>(pl + y * PC)[x];
  }
  TRACE(4, 15);
}

// ---------------------------------------------------------------------------
// k_gather: force interpolation, one atom per thread in sorted order.
// ---------------------------------------------------------------------------
template <class P, int K, int ORDER, bool BATCH>
__global__ __launch_bounds__(kGatherThreads) void k_gather(Args a_in, BatchArgs bt) {
  const Args a = BATCH ? *bt.sys[blockIdx.y] : a_in;
  using T = typename P::real;
  using Rec = typename P::rec;
  constexpr int PP = phi_pitch_of(K, ORDER);
  TRACE(5, 0);
  const int t = blockIdx.x * kGatherThreads + threadIdx.x;
  if (t >= a.N) return;
  const Rec r = reinterpret_cast<const Rec*>(a.ws + a.lay.rec)[t];
  const double qi = a.q[r.idx];
  const T* phi = reinterpret_cast<const T*>(a.ws + a.lay.phi);
  const int gx = r.g & 1023, gy = (r.g >> 10) & 1023, gz = (r.g >> 20) & 1023;
  T thx[ORDER], thy[ORDER], thz[ORDER], dthx[ORDER], dthy[ORDER], dthz[ORDER];
  bspline<ORDER>(r.w[0], thx, dthx);
  bspline<ORDER>(r.w[1], thy, dthy);
  bspline<ORDER>(r.w[2], thz, dthz);
  T sx = 0, sy = 0, sz = 0;
#pragma unroll
  for (int jz = 0; jz < ORDER; ++jz) {
    int zz = gz - ORDER + 1 + jz;
    if (zz < 0) zz += K;
#pragma unroll
    for (int jy = 0; jy < ORDER; ++jy) {
      int yy = gy - ORDER + 1 + jy;
      if (yy < 0) yy += K;
      const T* row = phi + ((size_t)zz * K + yy) * PP + gx;
      T s0 = 0, s1 = 0;
#pragma unroll
      for (int jx = 0; jx < ORDER; ++jx) {
        const T v = row[jx];
        s0 += thx[jx] * v;
        s1 += dthx[jx] * v;
      }
      sx += thy[jy] * thz[jz] * s1;
      sy += dthy[jy] * thz[jz] * s0;
      sz += thy[jy] * dthz[jz] * s0;
    }
  }
  const int idx = r.idx;
  const double qk = -qi * (double)K;
  const double f[3] = {qk * a.invL[0] * (double)sx, qk * a.invL[1] * (double)sy,
                       qk * a.invL[2] * (double)sz};
  double* out = a.forces + 3 * (size_t)idx;
  if (a.accumulate) {
    out[0] += f[0];
    out[1] += f[1];
    out[2] += f[2];
  } else {
    out[0] = f[0];
    out[1] = f[1];
    out[2] = f[2];
  }
  TRACE(5, 15);
}

__global__ void k_clear_flags(unsigned* ctrl) {
  if (threadIdx.x == 0) ctrl[0] = 0u;
}

// ---------------------------------------------------------------------------
// Host-side dispatch over (precision, K, order).
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
  if (t.start != nullptr)
    hipExtLaunchKernelGGL(kernel, grid, block, (uint32_t)lds, s, t.start, t.stop, 0u, a, b);
  else
    kernel<<<grid, block, lds, s>>>(a, b);
  return hipGetLastError();
}

// A launch that is skipped still closes its timing window.
static hipError_t skip(hipStream_t s, const Timing& t) {
  if (t.start == nullptr) return hipSuccess;
  hipError_t e = hipEventRecord(t.start, s);
  return e == hipSuccess ? hipEventRecord(t.stop, s) : e;
}

template <class F>
hipError_t with_prec(int prec, F&& f) {
  if (prec == PME_FP32_FIXED) return f(PFixed{});
  if (prec == PME_FP64) return f(PDouble{});
  return hipErrorInvalidValue;
}
template <class F>
hipError_t with_K(int K, F&& f) {
  switch (K) {
    case 16: return f(ic<16>{});
    case 24: return f(ic<24>{});
    case 32: return f(ic<32>{});
    case 48: return f(ic<48>{});
    case 64: return f(ic<64>{});
    case 96: return f(ic<96>{});
    case 128: return f(ic<128>{});
    default: return hipErrorInvalidValue;
  }
}
template <class F>
hipError_t with_order(int p, F&& f) {
  switch (p) {
    case 4: return f(ic<4>{});
    case 6: return f(ic<6>{});
    default: return hipErrorInvalidValue;
  }
}

bool grid_supported(int K) {
  return K == 16 || K == 24 || K == 32 || K == 48 || K == 64 || K == 96 || K == 128;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

bool layout_for(int K, int order, int max_atoms, int precision, Layout* lay) {
  if (!grid_supported(K) || (order != 4 && order != 6) || max_atoms < 0) return false;
  if (precision != PME_FP32_FIXED && precision != PME_FP64) return false;
  const bool fx = precision == PME_FP32_FIXED;
  const size_t real = fx ? 4 : 8, cpx = 2 * real;
  const size_t kh = (size_t)K / 2 + 1;
  const int nch = (max_atoms + kChunk - 1) / kChunk;
  const size_t nbins = 2 * (size_t)K * nq_of(K);
  Layout L{};
  size_t o = 0;
  L.ctrl = o;      o = align256(o + 64 * sizeof(unsigned));
  L.bsq = o;       o = align256(o + 3 * (size_t)K * sizeof(double));
  L.tw = o;        o = align256(o + (size_t)K * cpx);
  L.cnt = o;       o = align256(o + (size_t)nch * nbins * 2 * sizeof(int));
  L.absq = o;      o = align256(o + (size_t)nch * sizeof(double));
  L.rec = o;       o = align256(o + (size_t)nch * kChunk * (fx ? sizeof(RecF) : sizeof(RecD)));
  L.spec = o;      o = align256(o + (size_t)K * K * kh * cpx);
  L.phi_pitch = phi_pitch_of(K, order);
  L.phi = o;       o = align256(o + (size_t)K * K * L.phi_pitch * real);
  L.xsplit = pencil_xsplit(K);
  L.pencil_blocks = K * L.xsplit;
  L.partial = o;   o = align256(o + (size_t)L.pencil_blocks * 8 * sizeof(double));
  L.dbg = o;       o = align256(o + (size_t)K * K * K * 8);
  L.args = o;      o = align256(o + sizeof(Args));
  L.total = o;
  L.n_chunks_max = nch;
  *lay = L;
  return true;
}

template <class P, int KK, int O, bool B>
hipError_t raise_lds_limits() {
  const hipFuncAttribute attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  hipError_t e = hipFuncSetAttribute((const void*)k_spread_x<P, KK, O, B>, attr,
                                     (int)spread_lds_bytes<P, KK>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_fft_y<P, KK, B>, attr, (int)fft_y_lds_bytes<P, KK>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_inv_xy<P, KK, O, B>, attr, (int)inv_lds_bytes<P, KK>());
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_pencil<P, KK, B>, attr, (int)pencil_lds_bytes<P, KK>());
  return e;
}

hipError_t prepare_kernels(int K, int order, int precision) {
  return with_prec(precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        hipError_t e = raise_lds_limits<P, KK, O, false>();
        return e == hipSuccess ? raise_lds_limits<P, KK, O, true>() : e;
      });
    });
  });
}

template <class F>
hipError_t with_batch(const BatchArgs* bt, F&& f) {
  if (bt != nullptr) return f(std::true_type{});
  return f(std::false_type{});
}

hipError_t launch_bin(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  if (a.n_chunks == 0) return skip(s, t);
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_batch(bt, [&](auto bc) {
      constexpr bool B = decltype(bc)::value;
      return launch(k_bin<P, B>, dim3(a.n_chunks), dim3(kBinThreads), 0, s, t, a, bt);
    });
  });
}

hipError_t launch_spread_x(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(a.order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        return with_batch(bt, [&](auto bc) {
          constexpr bool B = decltype(bc)::value;
          return launch(k_spread_x<P, KK, O, B>, dim3(KK * nq_of(KK)), dim3(kSpreadThreads),
                        spread_lds_bytes<P, KK>(), s, t, a, bt);
        });
      });
    });
  });
}

hipError_t launch_fft_y(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_batch(bt, [&](auto bc) {
        constexpr bool B = decltype(bc)::value;
        const int blocks = KK + (P::fixed ? 1 : 0);
        return launch(k_fft_y<P, KK, B>, dim3(blocks), dim3(kPlaneThreads),
                      fft_y_lds_bytes<P, KK>(), s, t, a, bt);
      });
    });
  });
}

hipError_t launch_pencil(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_batch(bt, [&](auto bc) {
        constexpr bool B = decltype(bc)::value;
        return launch(k_pencil<P, KK, B>, dim3(KK * pencil_xsplit(KK)), dim3(kPencilThreads),
                      pencil_lds_bytes<P, KK>(), s, t, a, bt);
      });
    });
  });
}

hipError_t launch_reduce_ev(const Args& a, hipStream_t s) {
  k_reduce_ev<<<dim3(1), dim3(kPlaneThreads), 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_inv(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(a.order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        return with_batch(bt, [&](auto bc) {
          constexpr bool B = decltype(bc)::value;
          const int blocks = KK + ((a.reduce_ev || B) ? 1 : 0);
          return launch(k_inv_xy<P, KK, O, B>, dim3(blocks), dim3(kPlaneThreads),
                        inv_lds_bytes<P, KK>(), s, t, a, bt);
        });
      });
    });
  });
}

hipError_t launch_gather(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  if (a.N == 0) return skip(s, t);
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(a.order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        return with_batch(bt, [&](auto bc) {
          constexpr bool B = decltype(bc)::value;
          const int blocks = (a.N + kGatherThreads - 1) / kGatherThreads;
          return launch(k_gather<P, KK, O, B>, dim3(blocks), dim3(kGatherThreads), 0, s, t, a, bt);
        });
      });
    });
  });
}

hipError_t launch_clear_flags(const Args& a, hipStream_t s) {
  k_clear_flags<<<dim3(1), dim3(64), 0, s>>>(reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl));
  return hipGetLastError();
}

}  // namespace spme

#ifdef SPME_TRACE
// Trace builds only: point the phase trace at a device buffer of
// 6 * 1024 * 16 uint64 (or NULL to stop tracing).
extern "C" int spme_trace_set(void* buf) {
  unsigned long long* p = static_cast<unsigned long long*>(buf);
  return hipMemcpyToSymbol(HIP_SYMBOL(spme::g_trace), &p, sizeof(p)) == hipSuccess ? 0 : 5;
}
#endif
