// HIP kernels of the SPME reciprocal-space step for gfx950 (CDNA4).
//
// One step is five launches on one stream:
//   k_bin        fractional coordinates, base grid index and offsets of each
//                atom; per-chunk counting sort of the atoms by the z index of
//                their base point (the GPU counterpart of the paper's atom
//                reordering for hazard suppression, §III.A.1 / §V.C)
//   k_spread_fwd one z-plane per workgroup: every atom whose B-spline support
//                covers the plane adds its p x p contributions into an LDS
//                plane (64-bit fixed point: integer adds commute, so the grid
//                is bit-identical whatever the order), then the plane is
//                transformed along x (real-to-complex) and y in LDS and
//                written out as half-spectrum rows (§III.A.2: "each slab runs
//                independently to compute X and Y transforms")
//   k_pencil     one y row (or half of it) per workgroup: z transforms,
//                multiplication by the influence function with FP64 energy
//                and virial partials, inverse z transforms (§III.A.2: "Z
//                direction transforms, multiply by Green's function data,
//                compute Z^-1 transforms"); the last workgroup reduces the
//                partials in a fixed order
//   k_inv_xy     one z-plane per workgroup: inverse y and complex-to-real x
//                transforms, potential rows written with a (p-1)-point wrap
//                halo so interpolation reads contiguous runs
//   k_gather     one atom per thread: B-spline weights and derivatives, p^3
//                potential reads, forces scattered back to the caller's atom
//                order (§III.A.3)
// The paper's two all-to-all corner turns become the HBM round trips between
// plane and pencil passes.
#include <type_traits>

#include "spme_device.h"
#include "spme_internal.h"
#include "../../include/spme.h"

namespace spme {

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

// Row pitch of the LDS plane in 8-byte units.  Fixed point: K int64 values
// per row (the half spectrum of K/2+1 float2 fits in place).  FP64: room for
// K/2+1 double2.  One extra unit of padding skews rows across LDS banks.
template <class P>
__host__ __device__ constexpr int plane_pitch(int K) { return P::fixed ? K + 1 : K + 4; }
__host__ __device__ constexpr int pencil_xsplit(int K) { return K >= 32 ? 2 : 1; }
__host__ __device__ constexpr int phi_pitch_of(int K, int order) { return (K + order - 1 + 3) / 4 * 4; }

// a[i] for a register array and a lane-varying i, written as a masked sum
// (a[i] + exact zeros) so the array stays in registers.
template <int P, typename T>
__device__ __forceinline__ T pick(const T* a, int i) {
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

// Sum of one double over the block in a fixed order (wave shuffles, then the
// wave partials in order).  red needs blockDim/64 doubles.
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------
// k_bin: one chunk of kChunk atoms per workgroup.
// ---------------------------------------------------------------------------
template <class P>
__global__ __launch_bounds__(kBinThreads) void k_bin(Args a) {
  using Rec = typename P::rec;
  using T = typename P::real;
  __shared__ int hist[128];
  __shared__ int base[128];
  __shared__ double red[kBinThreads / 64];
  const int K = a.K;
  const int c = blockIdx.x, tid = threadIdx.x;
  int* cnt = reinterpret_cast<int*>(a.ws + a.lay.cnt) + (size_t)c * K;
  int* off = reinterpret_cast<int*>(a.ws + a.lay.off) + (size_t)c * K;
  Rec* rec = reinterpret_cast<Rec*>(a.ws + a.lay.rec) + (size_t)c * kChunk;
  unsigned* flags = reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl);
  for (int b = tid; b < K; b += kBinThreads) hist[b] = 0;
  __syncthreads();

  constexpr int APT = kChunk / kBinThreads;
  Rec r[APT];
  int bin[APT], rank[APT];
  double sabs = 0.0;
  bool bad = false;
#pragma unroll
  for (int t = 0; t < APT; ++t) {
    const int i = c * kChunk + t * kBinThreads + tid;
    bin[t] = -1;
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
        bad = true;
      }
      sabs += fabs(qi);
      r[t].g = g[0] | (g[1] << 10) | (g[2] << 20);
      r[t].w[0] = (T)w[0];
      r[t].w[1] = (T)w[1];
      r[t].w[2] = (T)w[2];
      r[t].q = (T)qi;
      r[t].idx = i;
      bin[t] = g[2];
      rank[t] = atomicAdd(&hist[g[2]], 1);
    }
  }
  if (bad) atomicOr(flags, PME_FLAG_NONFINITE);
  __syncthreads();
  {
    // K <= 128 bins: waves 0 and 1 scan 64 bins each; wave 1 adds wave 0's total
    __shared__ int wave0_total;
    const int lane = tid & 63, wave = tid >> 6;
    int h = 0, x = 0;
    if (wave < 2) {
      h = (tid < K) ? hist[tid] : 0;
      x = h;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      if (wave == 0 && lane == 63) wave0_total = x;
    }
    __syncthreads();
    if (wave < 2 && tid < K) {
      const int ex = x - h + (wave == 1 ? wave0_total : 0);
      base[tid] = ex;
      cnt[tid] = h;
      off[tid] = ex;
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < APT; ++t)
    if (bin[t] >= 0) rec[base[bin[t]] + rank[t]] = r[t];
  const double tot = block_sum(sabs, red);
  if (tid == 0) reinterpret_cast<double*>(a.ws + a.lay.absq)[c] = tot;
}

// ---------------------------------------------------------------------------
// k_spread_fwd: charge spreading of one z-plane, then x (R2C) and y FFTs.
// ---------------------------------------------------------------------------
template <class P, int K>
__host__ __device__ constexpr size_t spread_lds_bytes() {
  return (size_t)K * plane_pitch<P>(K) * 8 + (size_t)K * sizeof(cplx<typename P::real>) +
         (size_t)(2 * kPlaneThreads + 1 + 32) * sizeof(int) + 16 * sizeof(double);
}

template <class P, int K, int ORDER>
__global__ __launch_bounds__(kPlaneThreads) void k_spread_fwd(Args a) {
  using T = typename P::real;
  using Acc = typename P::acc;
  using Rec = typename P::rec;
  constexpr int M = K / 2, KH = K / 2 + 1;
  constexpr int PITCH = plane_pitch<P>(K);
  constexpr int PC = P::fixed ? PITCH : PITCH / 2;
  extern __shared__ __align__(16) unsigned char smem[];
  Acc* plane = reinterpret_cast<Acc*>(smem);
  cplx<T>* tw = reinterpret_cast<cplx<T>*>(smem + (size_t)K * PITCH * 8);
  double* red = reinterpret_cast<double*>(tw + K);
  int* segpre = reinterpret_cast<int*>(red + 16);
  int* segbeg = segpre + kPlaneThreads + 1;
  int* wsum = segbeg + kPlaneThreads;

  const int z = blockIdx.x, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < K; i += kPlaneThreads) tw[i] = twg[i];
  for (int i = tid; i < K * PITCH; i += kPlaneThreads) plane[i] = Acc(0);
  const int* cnt = reinterpret_cast<const int*>(a.ws + a.lay.cnt);
  const int* off = reinterpret_cast<const int*>(a.ws + a.lay.off);
  const Rec* rec = reinterpret_cast<const Rec*>(a.ws + a.lay.rec);
  const double scale = ldexp(1.0, a.frac_bits);
  __syncthreads();

  // --- spreading.  Plane z receives the atoms whose base z index b lies in
  // z .. z+p-1 (mod K); for b = z + j the plane is support point jz = p-1-j.
  // A segment is the run of such atoms inside one sorted chunk; segments are
  // taken kPlaneThreads at a time.  Each thread owns kItems (atom, plane)
  // items per pass and adds all p x p contributions of each; the items'
  // lookups and record loads are issued together so their latencies overlap.
  constexpr int kItems = 4;
  const int nseg = a.n_chunks * ORDER;
  for (int s0 = 0; s0 < nseg; s0 += kPlaneThreads) {
    const int ns = min(kPlaneThreads, nseg - s0);
    int len = 0;
    if (tid < ns) {
      const int seg = s0 + tid;
      const int c = seg / ORDER, j = seg - c * ORDER;
      int b = z + j;
      if (b >= K) b -= K;
      len = cnt[(size_t)c * K + b];
      segbeg[tid] = c * kChunk + off[(size_t)c * K + b];
    }
    int total;
    const int ex = block_exclusive_scan(len, wsum, &total);
    if (tid < ns) segpre[tid] = ex;
    if (tid == 0) segpre[ns] = total;
    __syncthreads();
    for (int it = 0; it < total; it += kItems * kPlaneThreads) {
      Rec r[kItems];
      int jz[kItems];
#pragma unroll
      for (int u = 0; u < kItems; ++u) {
        const int t = it + u * kPlaneThreads + tid;
        jz[u] = -1;
        if (t < total) {
          int lo = 0, hi = ns;  // segpre[lo] <= t < segpre[hi]
          while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (segpre[mid] <= t) lo = mid;
            else hi = mid;
          }
          r[u] = rec[segbeg[lo] + (t - segpre[lo])];
          jz[u] = ORDER - 1 - (s0 + lo) % ORDER;
        }
      }
#pragma unroll
      for (int u = 0; u < kItems; ++u) {
        if (jz[u] < 0) continue;
        const int gx = r[u].g & 1023, gy = (r[u].g >> 10) & 1023;
        T thx[ORDER], thy[ORDER], thz[ORDER];
        bspline<ORDER>(r[u].w[0], thx, (T*)nullptr);
        bspline<ORDER>(r[u].w[1], thy, (T*)nullptr);
        bspline<ORDER>(r[u].w[2], thz, (T*)nullptr);
        const T tz = pick<ORDER>(thz, jz[u]);
        int xs[ORDER];
#pragma unroll
        for (int jx = 0; jx < ORDER; ++jx) {
          int x = gx - ORDER + 1 + jx;
          xs[jx] = x < 0 ? x + K : x;
        }
#pragma unroll
        for (int jy = 0; jy < ORDER; ++jy) {
          int y = gy - ORDER + 1 + jy;
          if (y < 0) y += K;
          Acc* row = plane + y * PITCH;
          if constexpr (P::fixed) {
#pragma clang fp contract(off)
            const float cy = (r[u].q * tz) * thy[jy];  // product order z, y, x
#pragma unroll
            for (int jx = 0; jx < ORDER; ++jx) {
              const float cq = cy * thx[jx];
              atomicAdd(&row[xs[jx]], (unsigned long long)to_fixed(cq, scale));
            }
          } else {
            const T cy = r[u].q * tz * thy[jy];
#pragma unroll
            for (int jx = 0; jx < ORDER; ++jx) atomicAdd(&row[xs[jx]], cy * thx[jx]);
          }
        }
      }
    }
    __syncthreads();
  }

  // --- fixed-point headroom: sum |q| 2^F must stay below 2^52 so that every
  // grid value and its conversion to FP64 are exact.
  if (P::fixed && z == 0) {
    const double* absq = reinterpret_cast<const double*>(a.ws + a.lay.absq);
    double s = 0.0;
    for (int c = tid; c < a.n_chunks; c += kPlaneThreads) s += absq[c];
    s = block_sum(s, red);
    if (tid == 0 && s * scale >= 4503599627370496.0)
      atomicOr(reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl), PME_FLAG_OVERFLOW);
  }
  if (a.keep_grid) {
    Acc* dbg = reinterpret_cast<Acc*>(a.ws + a.lay.dbg) + (size_t)z * K * K;
    for (int i = tid; i < K * K; i += kPlaneThreads) dbg[i] = plane[(i / K) * PITCH + (i % K)];
  }
  __syncthreads();

  // --- x: real-to-complex, one row per group of fft_lanes(M) lanes.
  constexpr int TM = fft_lanes(M);
  for (int task = tid; task < K * TM; task += kPlaneThreads) {
    const int y = task / TM, l = task - y * TM;
    cplx<T>* row = reinterpret_cast<cplx<T>*>(plane + y * PITCH);
    if constexpr (P::fixed) {
      // int64 -> float in place: x_j at float slot j, so the row reads as the
      // packed complex sequence z_n = x_{2n} + i x_{2n+1}
      const double inv_scale = ldexp(1.0, -a.frac_bits);
      constexpr int PER = K / TM;
      float v[PER];
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const long long iv = (long long)plane[y * PITCH + l + i * TM];
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

  // --- y: complex FFT down each of the K/2+1 columns.
  constexpr int TK = fft_lanes(K);
  cplx<T>* pc = reinterpret_cast<cplx<T>*>(plane);
  for (int task = tid; task < KH * TK; task += kPlaneThreads) {
    const int x = task / TK, l = task - x * TK;
    fft_pencil<T, K, -1>(pc + x, PC, l, tw, 1);
  }
  __syncthreads();

  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.ws + a.lay.spec) + (size_t)z * K * KH;
  for (int i = tid; i < K * KH; i += kPlaneThreads) {
    const int y = i / KH, x = i - y * KH;
    spec[i] = pc[y * PC + x];
  }
}

// ---------------------------------------------------------------------------
// k_pencil: z FFT, influence function with energy/virial, inverse z FFT.
// ---------------------------------------------------------------------------
template <class P, int K>
__host__ __device__ constexpr size_t pencil_lds_bytes() {
  constexpr int KH = K / 2 + 1, XW = (KH + pencil_xsplit(K) - 1) / pencil_xsplit(K);
  return (size_t)K * (XW + 1) * sizeof(cplx<typename P::real>) +
         (size_t)K * sizeof(cplx<typename P::real>) + 3 * (size_t)K * sizeof(double) +
         8 * (kPencilThreads / 64) * sizeof(double) + 16;
}

template <class P, int K>
__global__ __launch_bounds__(kPencilThreads) void k_pencil(Args a) {
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
  __shared__ int is_last;

  const int tid = threadIdx.x;
  const int y = blockIdx.x / XS;
  const int x0 = (blockIdx.x - y * XS) * XW;
  const int xw = min(XW, KH - x0);
  cplx<T>* spec = reinterpret_cast<cplx<T>*>(a.ws + a.lay.spec);
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  const double* bsg = reinterpret_cast<const double*>(a.ws + a.lay.bsq);
  for (int i = tid; i < K; i += kPencilThreads) tw[i] = twg[i];
  for (int i = tid; i < 3 * K; i += kPencilThreads) bs[i] = bsg[i];
  for (int i = tid; i < K * XW; i += kPencilThreads) {
    const int zz = i / XW, xx = i - zz * XW;
    if (xx < xw) buf[zz * PW + xx] = spec[((size_t)zz * K + y) * KH + x0 + xx];
  }
  __syncthreads();

  constexpr int TK = fft_lanes(K);
  for (int task = tid; task < XW * TK; task += kPencilThreads) {
    const int xx = task / TK, l = task - xx * TK;
    if (xx < xw) fft_pencil<T, K, -1>(buf + xx, PW, l, tw, 1);
  }
  __syncthreads();

  // G(m) = c B(m) exp(-pi^2 |m|^2 / beta^2) / (pi V |m|^2); the half spectrum
  // counts every m1 = 1 .. K/2-1 twice (its Hermitian partner), m1 = 0 and
  // m1 = K/2 once.
  const double pref = a.coulomb / (PI * a.volume);
  const double fac = PI * PI / (a.beta * a.beta);
  const int my = (y <= K / 2) ? y : y - K;
  const double mvy = my * a.invL[1];
  const double ny = (2 * y == K) ? 0.0 : mvy;
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
      G = pref * bs[m1] * bs[K + y] * bs[2 * K + zz] * exp(-fac * msq) / msq;
      t = 2.0 * (1.0 + fac * msq) / msq;
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
  __syncthreads();

  for (int task = tid; task < XW * TK; task += kPencilThreads) {
    const int xx = task / TK, l = task - xx * TK;
    if (xx < xw) fft_pencil<T, K, 1>(buf + xx, PW, l, tw, 1);
  }
  __syncthreads();
  for (int i = tid; i < K * XW; i += kPencilThreads) {
    const int zz = i / XW, xx = i - zz * XW;
    if (xx < xw) spec[((size_t)zz * K + y) * KH + x0 + xx] = buf[zz * PW + xx];
  }

  // Energy/virial: fixed-order block sums, one partial row per workgroup;
  // the last workgroup to finish adds the rows in workgroup order.
  double* partial = reinterpret_cast<double*>(a.ws + a.lay.partial);
  double tot[7];
#pragma unroll
  for (int c = 0; c < 7; ++c) tot[c] = block_sum(acc[c], red);
  if (tid == 0) {
#pragma unroll
    for (int c = 0; c < 7; ++c) partial[blockIdx.x * 8 + c] = tot[c];
    __threadfence();
    unsigned* ticket = reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl) + 1;
    const unsigned prev =
        __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (is_last) {
    __threadfence();
    // every thread loads whole partial rows (in parallel), then the same
    // fixed-order block sum as above
    double r[7] = {0, 0, 0, 0, 0, 0, 0};
    for (unsigned b = tid; b < gridDim.x; b += kPencilThreads) {
#pragma unroll
      for (int c = 0; c < 7; ++c)
        r[c] += __hip_atomic_load(&partial[b * 8 + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    double sum[7];
#pragma unroll
    for (int c = 0; c < 7; ++c) sum[c] = block_sum(r[c], red);
    if (tid == 0) {
      if (a.ev != nullptr) {
#pragma unroll
        for (int c = 0; c < 7; ++c) a.ev[c] = sum[c];
      }
      unsigned* ticket = reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl) + 1;
      __hip_atomic_store(ticket, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// k_inv_xy: inverse y FFT and complex-to-real x FFT of one z-plane.
// ---------------------------------------------------------------------------
template <class P, int K>
__host__ __device__ constexpr size_t inv_lds_bytes() {
  return (size_t)K * (K / 2 + 2) * sizeof(cplx<typename P::real>) +
         (size_t)K * sizeof(cplx<typename P::real>);
}

template <class P, int K, int ORDER>
__global__ __launch_bounds__(kPlaneThreads) void k_inv_xy(Args a) {
  using T = typename P::real;
  constexpr int M = K / 2, KH = K / 2 + 1, PC = KH + 1;
  constexpr int PP = phi_pitch_of(K, ORDER);
  extern __shared__ __align__(16) unsigned char smem[];
  cplx<T>* pl = reinterpret_cast<cplx<T>*>(smem);
  cplx<T>* tw = pl + K * PC;
  const int z = blockIdx.x, tid = threadIdx.x;
  const cplx<T>* twg = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.tw);
  for (int i = tid; i < K; i += kPlaneThreads) tw[i] = twg[i];
  const cplx<T>* spec = reinterpret_cast<const cplx<T>*>(a.ws + a.lay.spec) + (size_t)z * K * KH;
  for (int i = tid; i < K * KH; i += kPlaneThreads) {
    const int y = i / KH, x = i - y * KH;
    pl[y * PC + x] = spec[i];
  }
  __syncthreads();

  constexpr int TK = fft_lanes(K);
  for (int task = tid; task < KH * TK; task += kPlaneThreads) {
    const int x = task / TK, l = task - x * TK;
    fft_pencil<T, K, 1>(pl + x, PC, l, tw, 1);
  }
  __syncthreads();

  constexpr int TM = fft_lanes(M);
  for (int task = tid; task < K * TM; task += kPlaneThreads) {
    const int y = task / TM, l = task - y * TM;
    cplx<T>* row = pl + y * PC;
    c2r_pre<T, K>(row, l, tw);
    fft_pencil<T, M, 1>(row, 1, l, tw, 2);
  }
  __syncthreads();

  T* phi = reinterpret_cast<T*>(a.ws + a.lay.phi) + (size_t)z * K * PP;
  for (int i = tid; i < K * PP; i += kPlaneThreads) {
    const int y = i / PP, xh = i - y * PP;
    int x = xh - (ORDER - 1);
    if (x < 0) x += K;
    if (x >= K) x -= K;
    phi[i] = reinterpret_cast<const T*>(pl + y * PC)[x];
  }
}

// ---------------------------------------------------------------------------
// k_gather: force interpolation, one atom per thread in sorted order.
// ---------------------------------------------------------------------------
template <class P, int K, int ORDER>
__global__ __launch_bounds__(kGatherThreads) void k_gather(Args a) {
  using T = typename P::real;
  using Rec = typename P::rec;
  constexpr int PP = phi_pitch_of(K, ORDER);
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
}

__global__ void k_clear_flags(unsigned* ctrl) {
  if (threadIdx.x == 0) ctrl[0] = 0u;
}

// ---------------------------------------------------------------------------
// Host-side dispatch over (precision, K, order).
// ---------------------------------------------------------------------------
template <int V>
using ic = std::integral_constant<int, V>;

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
  Layout L{};
  size_t o = 0;
  L.ctrl = o;      o = align256(o + 64 * sizeof(unsigned));
  L.bsq = o;       o = align256(o + 3 * (size_t)K * sizeof(double));
  L.tw = o;        o = align256(o + (size_t)K * cpx);
  L.cnt = o;       o = align256(o + (size_t)nch * K * sizeof(int));
  L.off = o;       o = align256(o + (size_t)nch * K * sizeof(int));
  L.absq = o;      o = align256(o + (size_t)nch * sizeof(double));
  L.rec = o;       o = align256(o + (size_t)nch * kChunk * (fx ? sizeof(RecF) : sizeof(RecD)));
  L.spec = o;      o = align256(o + (size_t)K * K * kh * cpx);
  L.phi_pitch = phi_pitch_of(K, order);
  L.phi = o;       o = align256(o + (size_t)K * K * L.phi_pitch * real);
  L.xsplit = pencil_xsplit(K);
  L.pencil_blocks = K * L.xsplit;
  L.partial = o;   o = align256(o + (size_t)L.pencil_blocks * 8 * sizeof(double));
  L.dbg = o;       o = align256(o + (size_t)K * K * K * 8);
  L.total = o;
  L.n_chunks_max = nch;
  *lay = L;
  return true;
}

hipError_t prepare_kernels(int K, int order, int precision) {
  return with_prec(precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        hipError_t e = hipFuncSetAttribute((const void*)k_spread_fwd<P, KK, O>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)spread_lds_bytes<P, KK>());
        if (e != hipSuccess) return e;
        e = hipFuncSetAttribute((const void*)k_inv_xy<P, KK, O>,
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)inv_lds_bytes<P, KK>());
        if (e != hipSuccess) return e;
        return hipFuncSetAttribute((const void*)k_pencil<P, KK>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)pencil_lds_bytes<P, KK>());
      });
    });
  });
}

hipError_t launch_bin(const Args& a, hipStream_t s) {
  if (a.n_chunks == 0) return hipSuccess;
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    k_bin<P><<<dim3(a.n_chunks), dim3(kBinThreads), 0, s>>>(a);
    return hipGetLastError();
  });
}

hipError_t launch_spread_fwd(const Args& a, hipStream_t s) {
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(a.order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        constexpr size_t lds = spread_lds_bytes<P, KK>();
        k_spread_fwd<P, KK, O><<<dim3(KK), dim3(kPlaneThreads), lds, s>>>(a);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_pencil(const Args& a, hipStream_t s) {
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      constexpr size_t lds = pencil_lds_bytes<P, KK>();
      k_pencil<P, KK><<<dim3(KK * pencil_xsplit(KK)), dim3(kPencilThreads), lds, s>>>(a);
      return hipGetLastError();
    });
  });
}

hipError_t launch_inv(const Args& a, hipStream_t s) {
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(a.order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        constexpr size_t lds = inv_lds_bytes<P, KK>();
        k_inv_xy<P, KK, O><<<dim3(KK), dim3(kPlaneThreads), lds, s>>>(a);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_gather(const Args& a, hipStream_t s) {
  if (a.N == 0) return hipSuccess;
  return with_prec(a.precision, [&](auto pt) {
    using P = decltype(pt);
    return with_K(a.K, [&](auto kc) {
      constexpr int KK = decltype(kc)::value;
      return with_order(a.order, [&](auto oc) {
        constexpr int O = decltype(oc)::value;
        const int blocks = (a.N + kGatherThreads - 1) / kGatherThreads;
        k_gather<P, KK, O><<<dim3(blocks), dim3(kGatherThreads), 0, s>>>(a);
        return hipGetLastError();
      });
    });
  });
}

hipError_t launch_clear_flags(const Args& a, hipStream_t s) {
  k_clear_flags<<<dim3(1), dim3(64), 0, s>>>(reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl));
  return hipGetLastError();
}

}  // namespace spme
