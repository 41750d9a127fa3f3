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
//   k_rs_count   wrap each atom into the cell, count atoms per cell; sum q^2
//                per workgroup (self term)
//   k_rs_scan    one workgroup: exclusive prefix sum of the counts
//   k_rs_fill    atoms into cell order (position, charge, original index)
//   k_rs_pairs   one cell per workgroup: its atoms, two threads each, against
//                the atoms of the 27 neighbour cells staged in LDS with their
//                periodic shifts applied; then each atom's excluded
//                partners; forces to the caller's order
//   k_rs_reduce  energies from the per-workgroup rows, in a fixed order
// Arithmetic is FP64 throughout.  The order of atoms inside a cell depends
// on atomic ordering, so forces are reproducible to FP64 rounding, not bit
// for bit.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "spme_device.h"
#include "spme_internal.h"
#include "../../include/spme.h"

namespace spme {
namespace {

constexpr int kRsThreads = 256;     // threads of a cell workgroup
constexpr int kRsHome = kRsThreads / 2;  // home atoms per pass (two threads each)
constexpr int kRsStage = 2048;      // neighbour atoms staged in LDS per pass
constexpr int kRsCountThreads = 256;
constexpr int kRsScanThreads = 1024;

struct RsArgs {
  int N, nc[3], ncell, n_count_blocks;
  double L[3], invL[3], cell_inv[3];
  double beta, rc2, rcut, coulomb;
  const double* pos;
  const double* q;
  const int* excl_off;  // may be null
  const int* excl_idx;
  double* forces;
  int accumulate;
  double* energies;
  // workspace
  unsigned* count;      // [ncell]
  unsigned* start;      // [ncell + 1]
  unsigned* cursor;     // [ncell]
  double4* rec;         // [N] wrapped position and charge, in cell order
  int* ridx;            // [N] original index, in cell order
  double* rows;         // [ncell][2] pair and exclusion energies; then [n_count_blocks] q^2 sums
};

__device__ __forceinline__ double wrap(double x, double L, double invL) {
  double s = x - L * floor(x * invL);
  if (s >= L) s -= L;  // rounding at the upper edge
  if (s < 0.0) s = 0.0;
  return s;
}

__device__ __forceinline__ int cell_of(const RsArgs& a, double x, double y, double z) {
  int c[3];
  const double w[3] = {x, y, z};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    c[d] = (int)(w[d] * a.cell_inv[d]);
    if (c[d] >= a.nc[d]) c[d] = a.nc[d] - 1;
    if (c[d] < 0) c[d] = 0;
  }
  return (c[2] * a.nc[1] + c[1]) * a.nc[0] + c[0];
}

__global__ __launch_bounds__(256) void k_rs_zero(RsArgs a) {
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < a.ncell; c += gridDim.x * blockDim.x)
    a.count[c] = 0u;
}

__global__ __launch_bounds__(kRsCountThreads) void k_rs_count(RsArgs a) {
  __shared__ double wred[16 * 8];
  const int i = blockIdx.x * kRsCountThreads + threadIdx.x;
  double v[1] = {0.0};
  if (i < a.N) {
    const double x = wrap(a.pos[3 * (size_t)i], a.L[0], a.invL[0]);
    const double y = wrap(a.pos[3 * (size_t)i + 1], a.L[1], a.invL[1]);
    const double z = wrap(a.pos[3 * (size_t)i + 2], a.L[2], a.invL[2]);
    atomicAdd(&a.count[cell_of(a, x, y, z)], 1u);
    v[0] = a.q[i] * a.q[i];
  }
  block_sums<1>(v, wred);
  if (threadIdx.x == 15) a.rows[2 * (size_t)a.ncell + blockIdx.x] = v[0];
}

// Exclusive prefix sum of the counts by one workgroup, in chunks of its size.
__global__ __launch_bounds__(kRsScanThreads) void k_rs_scan(RsArgs a) {
  __shared__ unsigned wsum[kRsScanThreads / 64];
  __shared__ unsigned carry;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) carry = 0u;
  __syncthreads();
  for (int c0 = 0; c0 < a.ncell; c0 += kRsScanThreads) {
    const int c = c0 + tid;
    const unsigned v = c < a.ncell ? a.count[c] : 0u;
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
    if (c < a.ncell) {
      a.start[c] = before + x - v;
      a.cursor[c] = before + x - v;
    }
    __syncthreads();
    if (tid == kRsScanThreads - 1) carry = before + x;
    __syncthreads();
  }
  if (tid == 0) a.start[a.ncell] = carry;
}

__global__ __launch_bounds__(256) void k_rs_fill(RsArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= a.N) return;
  const double x = wrap(a.pos[3 * (size_t)i], a.L[0], a.invL[0]);
  const double y = wrap(a.pos[3 * (size_t)i + 1], a.L[1], a.invL[1]);
  const double z = wrap(a.pos[3 * (size_t)i + 2], a.L[2], a.invL[2]);
  const unsigned slot = atomicAdd(&a.cursor[cell_of(a, x, y, z)], 1u);
  a.rec[slot] = make_double4(x, y, z, a.q[i]);
  a.ridx[slot] = i;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_pairs(RsArgs a) {
  __shared__ double4 stage[kRsStage];
  __shared__ int sidx[kRsStage];
  __shared__ int nb_start[27], nb_pre[28];
  __shared__ double nb_shift[27][3];
  __shared__ double fpart[kRsHome][3];
  __shared__ double wred[16 * 8];
  const int tid = threadIdx.x;
  const int cell = blockIdx.x;
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
    nb_start[tid] = (int)a.start[nbc];
    nb_pre[tid + 1] = (int)(a.start[nbc + 1] - a.start[nbc]);
  }
  __syncthreads();
  if (tid == 0) {
    nb_pre[0] = 0;
    for (int k = 0; k < 27; ++k) nb_pre[k + 1] += nb_pre[k];
  }
  __syncthreads();
  const int total = nb_pre[27];
  const int h0 = (int)a.start[cell], h1 = (int)a.start[cell + 1];
  const double two_over_sqrtpi = 1.12837916709551257390;
  double e_pair = 0.0, e_excl = 0.0;
  // each home atom takes two threads, which split its candidates (even and
  // odd staged entries); their forces are added in a fixed order
  const int slot = tid % kRsHome, part = tid / kRsHome;
  for (int hb = h0; hb < h1; hb += kRsHome) {
    const int h = hb + slot;
    const bool mine = h < h1;
    double4 ri = make_double4(0.0, 0.0, 0.0, 0.0);
    int ii = -1;
    if (mine) {
      ri = a.rec[h];
      ii = a.ridx[h];
    }
    double f[3] = {0.0, 0.0, 0.0};
    for (int s0 = 0; s0 < total; s0 += kRsStage) {
      const int sn = min(kRsStage, total - s0);
      __syncthreads();
      for (int t = tid; t < sn; t += kRsThreads) {
        const int g = s0 + t;
        int k = 0;
        while (nb_pre[k + 1] <= g) ++k;
        const int src = nb_start[k] + (g - nb_pre[k]);
        const double4 r = a.rec[src];
        stage[t] = make_double4(r.x + nb_shift[k][0], r.y + nb_shift[k][1], r.z + nb_shift[k][2], r.w);
        sidx[t] = a.ridx[src];
      }
      __syncthreads();
      if (mine) {
        for (int t = part; t < sn; t += 2) {
          const double4 rj = stage[t];
          const double d[3] = {ri.x - rj.x, ri.y - rj.y, ri.z - rj.z};
          const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          if (r2 <= a.rc2 && sidx[t] != ii) {
            const double r = sqrt(r2), br = a.beta * r;
            const double ec = erfc(br) / r;
            const double qq = a.coulomb * ri.w * rj.w;
            e_pair += 0.5 * qq * ec;
            const double g = qq * (ec + two_over_sqrtpi * a.beta * exp(-br * br)) / r2;
#pragma unroll
            for (int c = 0; c < 3; ++c) f[c] += g * d[c];
          }
        }
      }
    }
    if (mine && part == 0 && a.excl_off != nullptr) {
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
        for (int c = 0; c < 3; ++c) f[c] += g * d[c];
      }
    }
    __syncthreads();
    if (part == 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) fpart[slot][c] = f[c];
    }
    __syncthreads();
    if (mine && part == 0) {
      double* out = a.forces + 3 * (size_t)ii;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double fc = f[c] + fpart[slot][c];
        out[c] = a.accumulate ? out[c] + fc : fc;
      }
    }
  }
  double v[2] = {e_pair, e_excl};
  block_sums<2>(v, wred);
  if (tid == 15) {
    a.rows[2 * (size_t)cell] = v[0];
    a.rows[2 * (size_t)cell + 1] = v[1];
  }
}

// Energies in a fixed order by one wavefront: E_real, E_self, E_excl.
__global__ __launch_bounds__(64) void k_rs_reduce(RsArgs a) {
  double v[3] = {0.0, 0.0, 0.0};
  for (int r = threadIdx.x; r < a.ncell; r += 64) {
    v[0] += a.rows[2 * (size_t)r];
    v[2] += a.rows[2 * (size_t)r + 1];
  }
  for (int r = threadIdx.x; r < a.n_count_blocks; r += 64) v[1] += a.rows[2 * (size_t)a.ncell + r];
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
  L.count = o;   o = align256(o + (size_t)max_cells * sizeof(unsigned));
  L.start = o;   o = align256(o + ((size_t)max_cells + 1) * sizeof(unsigned));
  L.cursor = o;  o = align256(o + (size_t)max_cells * sizeof(unsigned));
  L.rec = o;     o = align256(o + (size_t)max_atoms * sizeof(double4));
  L.ridx = o;    o = align256(o + (size_t)max_atoms * sizeof(int));
  L.rows = o;    o = align256(o + (2 * (size_t)max_cells + nblk) * sizeof(double));
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
  k_rs_zero<<<dim3((a.ncell + 255) / 256), dim3(256), 0, s>>>(a);
  if (N > 0) {
    k_rs_count<<<dim3(a.n_count_blocks), dim3(kRsCountThreads), 0, s>>>(a);
  }
  k_rs_scan<<<dim3(1), dim3(kRsScanThreads), 0, s>>>(a);
  if (N > 0) k_rs_fill<<<dim3(nb), dim3(256), 0, s>>>(a);
  k_rs_pairs<<<dim3(a.ncell), dim3(kRsThreads), 0, s>>>(a);
  k_rs_reduce<<<dim3(1), dim3(64), 0, s>>>(a);
  return hipGetLastError() == hipSuccess ? PME_OK : PME_EDEVICE;
}

}  // extern "C"
