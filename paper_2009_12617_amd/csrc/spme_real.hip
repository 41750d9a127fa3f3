// Real-space part of the Ewald electrostatics on gfx950: the erfc-screened
// pair sum within a cutoff, the self term and the exclusion correction --
// the short-range work that the paper's system runs beside the long-range
// pipeline (§II, §V.A), so that reciprocal + real + self + exclusions give
// the full Ewald energy and forces.
//
// One evaluation is six launches on one stream, all over a cell grid of at
// least three cells of edge >= rcut per axis (so the 27 neighbour cells of
// a cell are distinct and minimum-image pairs within rcut are found once):
//   k_rs_zero    clear the cell counts
//   k_rs_count   wrap each atom into its cell, count atoms per (cell, octant); sum q^2
//                per workgroup (self term)
//   k_rs_scan    one workgroup: exclusive prefix sum of the counts
//   k_rs_fill    atoms into (cell, octant) order (position, charge, original index)
//   k_rs_pairs   kRsBlocks workgroups per cell: its atoms, 2 to 8 lanes each, against
//                the atoms of the 27 neighbour cells that lie within the
//                cutoff of the home atoms' bounding box, staged in LDS with
//                their periodic shifts applied; pairs inside the cutoff are queued
//                per wavefront and evaluated in batches of 64; then each
//                atom's excluded partners; forces to the caller's order
//   k_rs_reduce  energies from the per-workgroup rows, in a fixed order
// Arithmetic is FP64 throughout.  The order of atoms inside a cell and of
// the force additions depends on atomic ordering, so forces are
// reproducible to FP64 rounding, not bit for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "spme_device.h"
#include "spme_internal.h"
#include "../../include/spme.h"

namespace spme {
namespace {

constexpr int kRsThreads = 128;     // threads of a pair workgroup (two wavefronts)
constexpr int kRsHome = kRsThreads / 2;  // most home atoms per pass (two lanes each)
constexpr int kRsMaxSplit = 8;      // most lanes sharing one home atom's candidates
constexpr int kRsBlocks = 2;        // pair workgroups per cell (each a half of its atoms, in passes)
constexpr int kRsStage = 512;       // neighbour atoms staged in LDS per pass (< 2^24)
constexpr int kRsUnroll = 4;        // candidates each lane tests per step
constexpr int kRsPer = 4;           // neighbour atoms each thread reads per staging pass
static_assert(kRsStage % (kRsMaxSplit * kRsUnroll) == 0, "the padded stage must fit");
static_assert(kRsPer * kRsThreads >= kRsStage, "one staging pass reads the whole stage");
constexpr int kRsQueue = 512;       // ring of queued pairs per wavefront (>= 64 + 64 kRsUnroll, 2^n)
static_assert((kRsQueue & (kRsQueue - 1)) == 0 && kRsQueue >= 64 + 64 * kRsUnroll,
              "a wavefront's ring holds under 64 leftovers plus one step's hits");
constexpr int kRsCountThreads = 256;
constexpr int kRsCheb = 32;         // Chebyshev terms of exp(x^2) erfc(x)
constexpr int kRsChebShort = 24;    // terms enough for beta rcut <= kRsShortRange
constexpr double kRsShortRange = 3.2;  // 24 terms: <= 1.3e-14 relative up to here
constexpr double kRsMaxBetaRcut = 6.0;  // series error <= 2e-14 relative up to here
constexpr int kRsScanThreads = 1024;
constexpr int kRsScanPre = 8;       // chunks of counts the scan loads at once
// Atoms are ordered by cell and, inside a cell, by octant (x half fastest),
// so that the contiguous share of a cell's atoms each pair workgroup takes
// is compact in space (its bounding box, which bounds the candidates staged
// for it, is then smaller than the cell).
constexpr int kRsOct = 8;

struct RsArgs {
  int N, nc[3], ncell, n_count_blocks;
  int nrow;             // pair workgroups: ncell * kRsBlocks
  double L[3], invL[3], cell_inv[3];
  double beta, rc2, rcut, coulomb;
  double cheb[kRsCheb];  // exp(x^2) erfc(x) on [0, beta rcut] as a Chebyshev series
  int ncheb;             // terms the pair kernel uses: kRsChebShort or kRsCheb
  double cheb_scale;     // 2 / (beta rcut)
  const double* pos;
  const double* q;
  const int* excl_off;  // may be null
  const int* excl_idx;
  double* forces;
  int accumulate;
  double* energies;
  // workspace
  unsigned* count;      // [ncell * kRsOct]: per (cell, octant)
  unsigned* start;      // [ncell * kRsOct + 1]
  unsigned* cursor;     // [ncell * kRsOct]
  double4* rec;         // [N] wrapped position and charge, in cell order
  int* ridx;            // [N] original index, in cell order
  double* rows;         // [nrow][2] pair and exclusion energies; then [n_count_blocks] q^2 sums
};

__device__ __forceinline__ double wrap(double x, double L, double invL) {
  double s = x - L * floor(x * invL);
  if (s >= L) s -= L;  // rounding at the upper edge
  if (s < 0.0) s = 0.0;
  return s;
}

__device__ __forceinline__ int cell_of(const RsArgs& a, double x, double y, double z) {
  // (cell, octant): cell index times kRsOct plus the octant bits x | y << 1 | z << 2
  int c[3], o = 0;
  const double w[3] = {x, y, z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double u = w[d] * a.cell_inv[d];
    c[d] = (int)u;
    if (c[d] >= a.nc[d]) c[d] = a.nc[d] - 1;
    if (c[d] < 0) c[d] = 0;
    o |= (u - c[d] >= 0.5 ? 1 : 0) << d;
  }
  return ((c[2] * a.nc[1] + c[1]) * a.nc[0] + c[0]) * kRsOct + o;
}

__global__ __launch_bounds__(256) void k_rs_zero(RsArgs a) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell * kRsOct; c += gridDim.x * blockDim.x)
    a.count[c] = 0u;
}

// Adds n to counter[c] once per distinct c among the lanes of the
// wavefront (lanes with c < 0 take no part) and returns each lane's slot:
// the counter's old value plus the number of lanes of the same c below it.
// Neighbouring atoms (the atoms of a molecule) usually share a cell, so this
// issues a fraction of the per-atom atomics on the contended counters.  The
// groups of equal c are found first (ballots only); then every group's
// first lane issues its atomic at once, so the wavefront waits for one
// atomic round trip, not one per group.
__device__ __forceinline__ unsigned wave_add(unsigned* counter, int c) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(c >= 0);
  int leader = lane;  // first lane of this lane's group
  unsigned n = 0u, below = 0u;
  while (todo != 0ull) {  // uniform over the wavefront
    const int first = __ffsll((long long)todo) - 1;
    const int cl = __builtin_amdgcn_readlane(c, first);  // first is uniform
    const unsigned long long same = __ballot(c == cl) & todo;
    if (c == cl) {
      leader = first;
      below = __builtin_amdgcn_mbcnt_hi((unsigned)(same >> 32),
                                        __builtin_amdgcn_mbcnt_lo((unsigned)same, 0u));
    }
    if (lane == first) n = (unsigned)__popcll(same);
    todo &= ~same;
  }
  unsigned base = 0u;
  if (c >= 0 && lane == leader) base = atomicAdd(&counter[c], n);
  return __shfl(base, leader, 64) + below;
}

__global__ __launch_bounds__(kRsCountThreads) void k_rs_count(RsArgs a) {
  __shared__ double wred[16 * 8];
  const int i = blockIdx.x * kRsCountThreads + threadIdx.x;
  double v[1] = {0.0};
  int c = -1;
  if (i < a.N) {
    const double x = wrap(a.pos[3 * (size_t)i], a.L[0], a.invL[0]);
    const double y = wrap(a.pos[3 * (size_t)i + 1], a.L[1], a.invL[1]);
    const double z = wrap(a.pos[3 * (size_t)i + 2], a.L[2], a.invL[2]);
    c = cell_of(a, x, y, z);
    v[0] = a.q[i] * a.q[i];
  }
  (void)wave_add(a.count, c);
  block_sums<1>(v, wred);
  if (threadIdx.x == 15) a.rows[2 * (size_t)a.nrow + blockIdx.x] = v[0];
}

// Exclusive prefix sum of the counts by one workgroup, in chunks of its size.
__global__ __launch_bounds__(kRsScanThreads) void k_rs_scan(RsArgs a) {
  // the counts of up to kRsScanPre chunks of kRsScanThreads are loaded at
  // once, then scanned chunk by chunk from registers
  __shared__ unsigned wsum[kRsScanThreads / 64];
  __shared__ unsigned carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0u;
  __syncthreads();
  const int nsub = a.ncell * kRsOct;
  for (int s0 = 0; s0 < nsub; s0 += kRsScanThreads * kRsScanPre) {
    unsigned pv[kRsScanPre];
#pragma unroll
    for (int i = 0; i < kRsScanPre; ++i) {
      const int c = s0 + i * kRsScanThreads + tid;
      pv[i] = c < nsub ? a.count[c] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kRsScanPre; ++i) {
      const int c0 = s0 + i * kRsScanThreads;
      if (c0 >= nsub) break;  // uniform
      const int c = c0 + tid;
      const unsigned v = pv[i];
      unsigned x = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const unsigned y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
      }
      if (lane == 63) wsum[wave] = x;
      __syncthreads();
      unsigned before = carry;
      for (int w = 0; w < wave; ++w) before += wsum[w];
      if (c < nsub) {
        a.start[c] = before + x - v;
        a.cursor[c] = before + x - v;
      }
      __syncthreads();
      if (tid == kRsScanThreads - 1) carry = before + x;
      __syncthreads();
    }
  }
  if (tid == 0) a.start[nsub] = carry;
}

__global__ __launch_bounds__(256) void k_rs_fill(RsArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double x = 0.0, y = 0.0, z = 0.0;
  int c = -1;
  if (i < a.N) {
    x = wrap(a.pos[3 * (size_t)i], a.L[0], a.invL[0]);
    y = wrap(a.pos[3 * (size_t)i + 1], a.L[1], a.invL[1]);
    z = wrap(a.pos[3 * (size_t)i + 2], a.L[2], a.invL[2]);
    c = cell_of(a, x, y, z);
  }
  const unsigned slot = wave_add(a.cursor, c);
  if (c < 0) return;
  a.rec[slot] = make_double4(x, y, z, a.q[i]);
  a.ridx[slot] = i;
}

// One candidate pair taken from a wavefront's queue: entry = (staged index
// << 7) | home slot.  Adds the pair's energy to e and its force on the home
// atom to hf (LDS atomics: a home atom's pairs are spread over lanes and
// wavefronts).  erfc(x) = exp(-x^2) erfcx(x), with erfcx = exp(x^2) erfc(x)
// from its Chebyshev series on [0, beta rcut] (Clenshaw's recurrence over NC
// terms, 24 up to beta rcut = 3.2 and 32 beyond; the coefficients uniform
// over the launch), so the exp the force needs is the
// only transcendental besides 1/r (hardware reciprocal square root and two
// Newton steps).
template <int NC>
__device__ __forceinline__ void rs_pair(const RsArgs& a, const double4* stage, const double4* home,
                                        double (*hf)[3], int entry, double& e) {
  const double two_over_sqrtpi = 1.12837916709551257390;
  const int t = entry >> 7, s = entry & 127;
  const double4 rj = stage[t], ri = home[s];
  const double d[3] = {ri.x - rj.x, ri.y - rj.y, ri.z - rj.z};
  // the home atom's own staged copy (and an atom on the same position) is
  // queued too, at distance exactly 0: it adds nothing
  const bool paired = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] > 0.0;
  const double r2 = paired ? d[0] * d[0] + d[1] * d[1] + d[2] * d[2] : 1.0;
  double rinv = __builtin_amdgcn_rsq(r2);
  rinv = rinv * fma(-0.5 * r2 * rinv, rinv, 1.5);
  rinv = rinv * fma(-0.5 * r2 * rinv, rinv, 1.5);
  const double br = a.beta * (r2 * rinv);
  const double ex = exp(-br * br);
  const double tc = fma(br, a.cheb_scale, -1.0), t2 = tc + tc;
  double b1 = 0.0, b2 = 0.0;
#pragma unroll
  for (int k = NC - 1; k >= 1; --k) {
    const double b0 = fma(t2, b1, a.cheb[k] - b2);
    b2 = b1;
    b1 = b0;
  }
  const double ec = ex * fma(tc, b1, a.cheb[0] - b2) * rinv;  // erfc(beta r) / r
  const double qq = paired ? a.coulomb * ri.w * rj.w : 0.0;
  e += 0.5 * qq * ec;
  const double g = qq * (ec + two_over_sqrtpi * a.beta * ex) * (rinv * rinv);
#pragma unroll
  for (int c = 0; c < 3; ++c) atomicAdd(&hf[s][c], g * d[c]);
}

template <int NC>
__global__ __launch_bounds__(kRsThreads, 3) void k_rs_pairs(RsArgs a) {
  __shared__ double4 stage[kRsStage];
  __shared__ int nb_start[27], nb_pre[28];
  __shared__ double nb_shift[27][3];
  __shared__ double4 home[kRsHome];
  __shared__ double hf[kRsHome][3];
  __shared__ int queue[kRsThreads / 64][kRsQueue];
  __shared__ double wred[16 * 8];
  __shared__ double hbox[6];                  // home pass bounding box: low x y z, high x y z
  __shared__ int kept[kRsThreads / 64];       // staged atoms kept per wavefront
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int cell = blockIdx.x, blk = blockIdx.y;
  const int cx = cell % a.nc[0], cy = (cell / a.nc[0]) % a.nc[1], cz = cell / (a.nc[0] * a.nc[1]);
  if (tid < 27) {
    // neighbour cell and the periodic shift that brings its atoms next to
    // this cell (at least three cells per axis: each neighbour appears once)
    const int dd[3] = {tid % 3 - 1, (tid / 3) % 3 - 1, tid / 9 - 1};
    const int cc[3] = {cx, cy, cz};
    int n3[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      int v = cc[d] + dd[d];
      double sh = 0.0;
      if (v < 0) {
        v += a.nc[d];
        sh = -a.L[d];
      } else if (v >= a.nc[d]) {
        v -= a.nc[d];
        sh = a.L[d];
      }
      n3[d] = v;
      nb_shift[tid][d] = sh;
    }
    const int nbc = (n3[2] * a.nc[1] + n3[1]) * a.nc[0] + n3[0];
    nb_start[tid] = (int)a.start[nbc * kRsOct];
    nb_pre[tid + 1] = (int)(a.start[(nbc + 1) * kRsOct] - a.start[nbc * kRsOct]);
  }
  __syncthreads();
  if (tid == 0) {
    nb_pre[0] = 0;
    for (int k = 0; k < 27; ++k) nb_pre[k + 1] += nb_pre[k];
  }
  __syncthreads();
  const int total = nb_pre[27];
  const int h0 = (int)a.start[cell * kRsOct], h1 = (int)a.start[(cell + 1) * kRsOct];
  const double two_over_sqrtpi = 1.12837916709551257390;
  double e_pair = 0.0, e_excl = 0.0;
  int* wq = queue[wave];
  // Home atoms of the cell (in octant order) dealt in contiguous chunks over
  // its kRsBlocks workgroups -- a half each for cells of up to 2 kRsHome
  // atoms -- in passes of at most kRsHome.  S lanes share a home atom (S = 2, 4 or 8,
  // the most that fit the workgroup: lane L takes home L mod nh and every
  // S-th candidate from L / nh), so a sparsely filled pass still spreads its
  // candidate tests over the whole workgroup.  Each lane tests its
  // candidates in step with the wavefront (every lane reads the same staged
  // atom); pairs inside the cutoff go to the wavefront's queue, and the erfc
  // work runs only on full batches of 64 queued pairs, one per lane.
  const int chunk = max(1, min(kRsHome, (h1 - h0 + kRsBlocks - 1) / kRsBlocks));
  for (int hb = h0 + blk * chunk; hb < h1; hb += kRsBlocks * chunk) {
    const int nh = min(chunk, h1 - hb);
    const int S = nh > kRsThreads / 4 ? 2 : nh > kRsThreads / 8 ? 4 : kRsMaxSplit;
    const bool active = tid < S * nh;
    const int slot = active ? tid % nh : 0, split = active ? tid / nh : 0;
    __syncthreads();  // the previous pass is done with home and hf
    if (tid < nh) {
      home[tid] = a.rec[hb + tid];
      hf[tid][0] = hf[tid][1] = hf[tid][2] = 0.0;
    }
    if (wave == 0) {  // the bounding box of this pass's home atoms (nh <= 64)
      const double4 h = a.rec[hb + min(tid, nh - 1)];
      double bx[6] = {h.x, h.y, h.z, h.x, h.y, h.z};
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          bx[c] = fmin(bx[c], __shfl_xor(bx[c], d));
          bx[3 + c] = fmax(bx[3 + c], __shfl_xor(bx[3 + c], d));
        }
      }
      if (tid == 0) {
#pragma unroll
        for (int c = 0; c < 6; ++c) hbox[c] = bx[c];
      }
    }
    // an idle lane sits far from every atom and never finds a pair
    double4 ri = make_double4(-1e30, -1e30, -1e30, 0.0);
    int ii = -1;
    if (active) {
      ri = a.rec[hb + slot];
      ii = a.ridx[hb + slot];
    }
    for (int s0 = 0; s0 < total; s0 += kRsStage) {
      // kRsStage neighbour atoms (with their periodic shifts) are read per
      // pass, kRsPer consecutive ones per thread, and only those within the
      // cutoff of the home atoms' bounding box are staged, in their original
      // order (a scan over the workgroup): no partner of a home atom inside
      // the cutoff is dropped (the box test is a lower bound of every
      // home-candidate distance, with a margin for its rounding)
      const int sr = min(kRsStage, total - s0);
      __syncthreads();
      double4 cand[kRsPer];
      unsigned keep = 0u;
      const int tb = tid * kRsPer;
      if (tb < sr) {
        const double lim = a.rc2 * (1.0 + 1e-12) + 1e-12;
        int k = 0;
#pragma unroll
        for (int j = 0; j < kRsPer; ++j) {
          const int g = s0 + tb + j;
          if (tb + j < sr) {
            while (nb_pre[k + 1] <= g) ++k;
            const double4 r = a.rec[nb_start[k] + (g - nb_pre[k])];
            cand[j] = make_double4(r.x + nb_shift[k][0], r.y + nb_shift[k][1], r.z + nb_shift[k][2], r.w);
            const double dx = fmax(fmax(hbox[0] - cand[j].x, cand[j].x - hbox[3]), 0.0);
            const double dy = fmax(fmax(hbox[1] - cand[j].y, cand[j].y - hbox[4]), 0.0);
            const double dz = fmax(fmax(hbox[2] - cand[j].z, cand[j].z - hbox[5]), 0.0);
            if (dx * dx + dy * dy + dz * dz <= lim) keep |= 1u << j;
          }
        }
      }
      const int c = __popc(keep);
      int inc = c;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(inc, d);
        if (lane >= d) inc += o;
      }
      if (lane == 63) kept[wave] = inc;
      __syncthreads();
      int sn = 0, o = inc - c;
#pragma unroll
      for (int w = 0; w < kRsThreads / 64; ++w) {
        if (w < wave) o += kept[w];
        sn += kept[w];
      }
#pragma unroll
      for (int j = 0; j < kRsPer; ++j)
        if (keep & (1u << j)) stage[o++] = cand[j];
      // padded to whole steps with atoms far away (never inside the cutoff);
      // kRsStage is a multiple of every step S * kRsUnroll
      const int snp = (sn + S * kRsUnroll - 1) / (S * kRsUnroll) * (S * kRsUnroll);
      for (int t = sn + tid; t < snp; t += kRsThreads) stage[t] = make_double4(1e30, 1e30, 1e30, 0.0);
      __syncthreads();
      if (wave * 64 >= S * nh) continue;  // no active lane in this wavefront
      // ring of queued pairs: head qh, length qn (uniform over the wavefront)
      int qh = 0, qn = 0;
      const int entry0 = (split << 7) | slot;
      for (int t0 = 0; t0 < sn; t0 += S * kRsUnroll) {
        // kRsUnroll candidates per lane, loads issued together
        double4 rj[kRsUnroll];
#pragma unroll
        for (int u = 0; u < kRsUnroll; ++u) rj[u] = stage[t0 + S * u + split];
#pragma unroll
        for (int u = 0; u < kRsUnroll; ++u) {
          // one compare per candidate: the home atom's own staged copy (at
          // distance exactly 0) is queued as well and adds nothing there
          const double d0 = ri.x - rj[u].x, d1 = ri.y - rj[u].y, d2 = ri.z - rj[u].z;
          const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
          const bool hit = r2 <= a.rc2;
          const unsigned long long m = __ballot(hit);
          if (hit) {
            const int below = (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                             __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
            wq[(qh + qn + below) & (kRsQueue - 1)] = entry0 + ((t0 + S * u) << 7);
          }
          qn += __popcll(m);
        }
        while (qn >= 64) {
          lds_order();
          rs_pair<NC>(a, stage, home, hf, wq[(qh + lane) & (kRsQueue - 1)], e_pair);
          qh += 64;
          qn -= 64;
        }
      }
      lds_order();
      if (lane < qn) rs_pair<NC>(a, stage, home, hf, wq[(qh + lane) & (kRsQueue - 1)], e_pair);
    }
    if (active && split == 0 && a.excl_off != nullptr) {
      // excluded partners: remove the erfc/r the pair sum took (inside the
      // cutoff) and the erf/r the reciprocal sum carries
      const double* pi = a.pos + 3 * (size_t)ii;
      for (int k = a.excl_off[ii]; k < a.excl_off[ii + 1]; ++k) {
        const int j = a.excl_idx[k];
        const double* pj = a.pos + 3 * (size_t)j;
        double d[3] = {pi[0] - pj[0], pi[1] - pj[1], pi[2] - pj[2]};
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] -= a.L[c] * rint(d[c] * a.invL[c]);
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double r = sqrt(r2);
        const double qq = a.coulomb * ri.w * a.q[j];
        double u, du;
        if (r2 <= a.rc2) {
          u = 1.0 / r;
          du = -1.0 / r2;
        } else {
          const double ef = erf(a.beta * r);
          u = ef / r;
          du = (two_over_sqrtpi * a.beta * exp(-a.beta * a.beta * r2) - ef / r) / r;
        }
        e_excl -= 0.5 * qq * u;
        const double g = qq * du / r;
#pragma unroll
        for (int c = 0; c < 3; ++c) atomicAdd(&hf[slot][c], g * d[c]);
      }
    }
    __syncthreads();
    if (tid < nh) {
      double* out = a.forces + 3 * (size_t)a.ridx[hb + tid];
#pragma unroll
      for (int c = 0; c < 3; ++c) out[c] = a.accumulate ? out[c] + hf[tid][c] : hf[tid][c];
    }
  }
  double v[2] = {e_pair, e_excl};
  block_sums<2>(v, wred);
  if (tid == 15) {
    const size_t row = (size_t)cell * kRsBlocks + blk;
    a.rows[2 * row] = v[0];
    a.rows[2 * row + 1] = v[1];
  }
}

// Energies in a fixed order by one wavefront: E_real, E_self, E_excl.
__global__ __launch_bounds__(64) void k_rs_reduce(RsArgs a) {
  // (unrolled so that the loads of several rows are in flight together;
  // the additions keep their row order)
  double v[3] = {0.0, 0.0, 0.0};
#pragma unroll 8
  for (int r = threadIdx.x; r < a.nrow; r += 64) {
    v[0] += a.rows[2 * (size_t)r];
    v[2] += a.rows[2 * (size_t)r + 1];
  }
#pragma unroll 8
  for (int r = threadIdx.x; r < a.n_count_blocks; r += 64) v[1] += a.rows[2 * (size_t)a.nrow + r];
  wave_sums<3>(v);
  if (threadIdx.x == 63) {
    a.energies[0] = v[0];
    a.energies[1] = -a.coulomb * a.beta * 0.56418958354775628695 * v[1];  // -c beta/sqrt(pi) sum q^2
    a.energies[2] = v[2];
  }
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct RsLayout {
  size_t count, start, cursor, rec, ridx, rows, total;
};

RsLayout rs_layout(int max_atoms, int max_cells) {
  const int nblk = (max_atoms + kRsCountThreads - 1) / kRsCountThreads;
  RsLayout L{};
  size_t o = 0;
  const size_t nsub = (size_t)max_cells * kRsOct;
  L.count = o;   o = align256(o + nsub * sizeof(unsigned));
  L.start = o;   o = align256(o + (nsub + 1) * sizeof(unsigned));
  L.cursor = o;  o = align256(o + nsub * sizeof(unsigned));
  L.rec = o;     o = align256(o + (size_t)max_atoms * sizeof(double4));
  L.ridx = o;    o = align256(o + (size_t)max_atoms * sizeof(int));
  L.rows = o;    o = align256(o + (2 * (size_t)max_cells * kRsBlocks + nblk) * sizeof(double));
  L.total = o;
  return L;
}

constexpr int kRsMaxAtoms = 1 << 26;
constexpr int kRsMaxCells = 1 << 20;

}  // namespace
}  // namespace spme

extern "C" {

size_t pme_real_workspace_bytes(int max_atoms, int max_cells) {
  if (max_atoms < 0 || max_atoms > spme::kRsMaxAtoms || max_cells < 27 ||
      max_cells > spme::kRsMaxCells)
    return 0;
  return spme::rs_layout(max_atoms, max_cells).total;
}

int pme_real(const double* pos, const double* q, int N, const double box[9], double beta,
             double rcut, double coulomb, const int* excl_off, const int* excl_idx, double* forces,
             int accumulate, double* energies, void* workspace, size_t workspace_bytes,
             int max_atoms, int max_cells, void* stream) {
  using namespace spme;
  if (box == nullptr || energies == nullptr || workspace == nullptr) return PME_EINVAL;
  if (N < 0 || N > max_atoms || (N > 0 && (pos == nullptr || q == nullptr || forces == nullptr)))
    return PME_EINVAL;
  if ((excl_off == nullptr) != (excl_idx == nullptr)) return PME_EINVAL;
  if (!(beta > 0.0) || !(rcut > 0.0) || !std::isfinite(beta) || !std::isfinite(rcut))
    return PME_EINVAL;
  if (beta * rcut > kRsMaxBetaRcut) return PME_EUNSUPPORTED;  // erfc(6) < 3e-17
  if (coulomb == 0.0) coulomb = 1.0;
  for (int i = 0; i < 9; ++i)
    if (!std::isfinite(box[i])) return PME_EINVAL;
  if (box[1] != 0.0 || box[2] != 0.0 || box[3] != 0.0 || box[5] != 0.0 || box[6] != 0.0 ||
      box[7] != 0.0)
    return PME_EUNSUPPORTED;  // the cell search assumes a diagonal box
  const double L[3] = {box[0], box[4], box[8]};
  if (!(L[0] > 0.0 && L[1] > 0.0 && L[2] > 0.0)) return PME_EINVAL;
  const size_t need = pme_real_workspace_bytes(max_atoms, max_cells);
  if (need == 0) return PME_EINVAL;
  if (workspace_bytes < need || (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
    return PME_EWORKSPACE;
  RsArgs a{};
  long long ncell = 1;
  for (int d = 0; d < 3; ++d) {
    a.nc[d] = (int)std::floor(L[d] / rcut);
    if (a.nc[d] < 3) return PME_EUNSUPPORTED;  // rcut must be <= L/3 along every axis
    ncell *= a.nc[d];
  }
  while (ncell > max_cells) {  // coarser cells (edge still >= rcut)
    int big = 0;
    for (int d = 1; d < 3; ++d)
      if (a.nc[d] > a.nc[big]) big = d;
    if (a.nc[big] <= 3) return PME_EWORKSPACE;
    ncell = ncell / a.nc[big] * (a.nc[big] - 1);
    a.nc[big] -= 1;
  }
  a.ncell = (int)ncell;
  a.nrow = (int)ncell * kRsBlocks;
  a.N = N;
  a.n_count_blocks = (N + kRsCountThreads - 1) / kRsCountThreads;
  for (int d = 0; d < 3; ++d) {
    a.L[d] = L[d];
    a.invL[d] = 1.0 / L[d];
    a.cell_inv[d] = a.nc[d] / L[d];
  }
  a.beta = beta;
  a.rcut = rcut;
  a.rc2 = rcut * rcut;
  // exp(x^2) erfc(x) on [0, X], X = beta rcut: Chebyshev coefficients from
  // its values at 64 Chebyshev nodes (a discrete cosine transform), the
  // first kRsCheb kept
  {
    const double X = beta * rcut;
    const double pi = 3.14159265358979323846;
    constexpr int kNodes = 64;
    double f[kNodes];
    for (int j = 0; j < kNodes; ++j) {
      const double x = 0.5 * X * (std::cos(pi * (j + 0.5) / kNodes) + 1.0);
      f[j] = std::erfc(x) * std::exp(x * x);
    }
    for (int k = 0; k < kRsCheb; ++k) {
      double c = 0.0;
      for (int j = 0; j < kNodes; ++j) c += f[j] * std::cos(pi * k * (j + 0.5) / kNodes);
      a.cheb[k] = (k == 0 ? 1.0 : 2.0) * c / kNodes;
    }
    a.cheb_scale = 2.0 / X;
    // a shorter range needs fewer terms (the coefficients of this entire
    // function fall off faster on a shorter interval)
    a.ncheb = X <= kRsShortRange ? kRsChebShort : kRsCheb;
  }
  a.coulomb = coulomb;
  a.pos = pos;
  a.q = q;
  a.excl_off = excl_off;
  a.excl_idx = excl_idx;
  a.forces = forces;
  a.accumulate = accumulate ? 1 : 0;
  a.energies = energies;
  const RsLayout W = rs_layout(max_atoms, max_cells);
  char* ws = static_cast<char*>(workspace);
  a.count = reinterpret_cast<unsigned*>(ws + W.count);
  a.start = reinterpret_cast<unsigned*>(ws + W.start);
  a.cursor = reinterpret_cast<unsigned*>(ws + W.cursor);
  a.rec = reinterpret_cast<double4*>(ws + W.rec);
  a.ridx = reinterpret_cast<int*>(ws + W.ridx);
  a.rows = reinterpret_cast<double*>(ws + W.rows);
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int nb = (N + 255) / 256;
  k_rs_zero<<<dim3((a.ncell * kRsOct + 255) / 256), dim3(256), 0, s>>>(a);
  if (N > 0) {
    k_rs_count<<<dim3(a.n_count_blocks), dim3(kRsCountThreads), 0, s>>>(a);
  }
  k_rs_scan<<<dim3(1), dim3(kRsScanThreads), 0, s>>>(a);
  if (N > 0) k_rs_fill<<<dim3(nb), dim3(256), 0, s>>>(a);
  if (a.ncheb == kRsChebShort)
    k_rs_pairs<kRsChebShort><<<dim3(a.ncell, kRsBlocks), dim3(kRsThreads), 0, s>>>(a);
  else
    k_rs_pairs<kRsCheb><<<dim3(a.ncell, kRsBlocks), dim3(kRsThreads), 0, s>>>(a);
  k_rs_reduce<<<dim3(1), dim3(64), 0, s>>>(a);
  return hipGetLastError() == hipSuccess ? PME_OK : PME_EDEVICE;
}

}  // extern "C"
