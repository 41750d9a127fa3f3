// C ABI of the SPME step: argument validation, workspace layout, plan tables
// and launch sequencing.  All device work is enqueued on the plan's stream;
// the library allocates no device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <algorithm>
#include <vector>

#include "../../include/spme.h"
#include "spme_internal.h"

using spme::Args;
using spme::Layout;

namespace {

constexpr int kMaxAtoms = 1 << 26;

struct TimedLaunch {
  int kernel;
  hipEvent_t start, stop;
};

// kSpread: binned and spread, bucket counts still live (a new spread must
// clear them first); kSolved: convolved, counts cleared; kDirty: a launch
// failed midway, counts unknown.
enum State { kCreated = 0, kSpread = 1, kSolved = 2, kDirty = 3 };

}  // namespace

struct pme_plan {
  int K1 = 0, K2 = 0, K3 = 0, order = 0, precision = 0, frac_bits = 32, max_atoms = 0;
  double beta = 0.0, coulomb = 1.0;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  Layout lay{};
  Args cur{};
  int state = kCreated;
  int keep_grid = 0;
  int grid_kept = 0;
  // host copies of the uploaded tables
  std::vector<double> bsq;
  std::vector<double> tw64;
  std::vector<float> tw32;
  // per-kernel timing
  int timing = 0;
  std::vector<hipEvent_t> event_pool;
  size_t event_next = 0;
  std::vector<TimedLaunch> pending;
  int timed_steps = 0;
  // arguments bound for batched runs (host copy of the device copy)
  Args bound{};
  int is_bound = 0;
};

namespace {

// Cardinal B-spline M_n at integer arguments 1..n-1 by the order recursion
// M_n(x) = [x M_{n-1}(x) + (n - x) M_{n-1}(x - 1)] / (n - 1).
double bspline_at(int n, double x) {
  if (n == 2) return (x >= 0.0 && x <= 2.0) ? 1.0 - std::fabs(x - 1.0) : 0.0;
  return (x * bspline_at(n - 1, x) + (n - x) * bspline_at(n - 1, x - 1.0)) / (n - 1);
}

// |b(m)|^2 = 1 / |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K)|^2 (even p: no zeros).
void moduli(int p, int K, double* out) {
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < K; ++m) {
    double re = 0.0, im = 0.0;
    for (int k = 0; k <= p - 2; ++k) {
      const double c = bspline_at(p, k + 1.0);
      const double ang = 2.0 * pi * (double)((long)m * k % K) / (double)K;
      re += c * std::cos(ang);
      im += c * std::sin(ang);
    }
    out[m] = 1.0 / (re * re + im * im);
  }
}

bool is_fin(double x) { return std::isfinite(x); }

int device_error(hipError_t e) { return e == hipSuccess ? PME_OK : PME_EDEVICE; }

hipEvent_t next_event(pme_plan* p) {
  if (p->event_next == p->event_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p->event_pool.push_back(e);
  }
  return p->event_pool[p->event_next++];
}

// Run one launch; with timing on, events are attached to the dispatch and
// queued for pme_kernel_times.
template <class F>
int timed(pme_plan* p, int kernel, F&& launch) {
  if (!p->timing) return device_error(launch(spme::Timing()));
  spme::Timing t;
  t.start = next_event(p);
  t.stop = next_event(p);
  if (!t.start || !t.stop) return PME_EDEVICE;
  if (launch(t) != hipSuccess) return PME_EDEVICE;
  p->pending.push_back({kernel, t.start, t.stop});
  return PME_OK;
}

}  // namespace

extern "C" {

int pme_version(void) { return 200; }

const char* pme_strerror(int code) {
  switch (code) {
    case PME_OK: return "ok";
    case PME_EINVAL: return "invalid argument";
    case PME_EUNSUPPORTED: return "unsupported parameters (grid, spline order or cell shape)";
    case PME_EWORKSPACE: return "workspace missing, misaligned or too small";
    case PME_EOVERFLOW: return "fixed-point headroom exceeded (sum |q| 2^F >= 2^51)";
    case PME_EDEVICE: return "HIP runtime error";
    case PME_ENONFINITE: return "non-finite position or charge";
    case PME_ESTATE: return "call out of order";
    default: return "unknown status";
  }
}

size_t pme_workspace_bytes(int K1, int K2, int K3, int order, int max_atoms, int precision) {
  if (max_atoms < 0 || max_atoms > kMaxAtoms) return 0;
  Layout L;
  if (!spme::layout_for(K1, K2, K3, order, max_atoms, precision, &L)) return 0;
  return L.total;
}

int pme_create(pme_plan** out, int K1, int K2, int K3, int order, double beta, int max_atoms,
               int precision, int frac_bits, double coulomb, void* workspace,
               size_t workspace_bytes, void* stream) {
  if (out == nullptr) return PME_EINVAL;
  *out = nullptr;
  if (K1 < 2 || K2 < 2 || K3 < 2 || order < 3 || !(beta > 0.0) || !is_fin(beta) ||
      max_atoms < 0 ||
      (precision != PME_FP64 && precision != PME_FP32_FIXED && precision != PME_FP32_FIXED_HALF &&
       precision != PME_FP32_FIXED_BF16) ||
      !is_fin(coulomb))
    return PME_EINVAL;
  if (frac_bits == 0) frac_bits = 32;
  if (frac_bits < 16 || frac_bits > 40) return PME_EINVAL;
  if (coulomb == 0.0) coulomb = 1.0;
  if (!spme::grid_supported(K1, K2, K3) || (order != 4 && order != 6) || max_atoms > kMaxAtoms)
    return PME_EUNSUPPORTED;
  Layout L;
  if (!spme::layout_for(K1, K2, K3, order, max_atoms, precision, &L)) return PME_EUNSUPPORTED;
  if (workspace == nullptr || workspace_bytes < L.total ||
      (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
    return PME_EWORKSPACE;

  pme_plan* p = new (std::nothrow) pme_plan();
  if (p == nullptr) return PME_EDEVICE;
  p->K1 = K1;
  p->K2 = K2;
  p->K3 = K3;
  p->order = order;
  p->precision = precision;
  p->frac_bits = frac_bits;
  p->max_atoms = max_atoms;
  p->beta = beta;
  p->coulomb = coulomb;
  p->ws = static_cast<char*>(workspace);
  p->ws_bytes = workspace_bytes;
  p->stream = static_cast<hipStream_t>(stream);
  p->lay = L;

  // Tables per axis, x then y then z: moduli |b_a(m)|^2 and twiddles
  // exp(-2 pi i k / K_a), rounded once from FP64.
  const int Ks[3] = {K1, K2, K3};
  const int ksum = K1 + K2 + K3;
  const double pi = 3.14159265358979323846;
  p->bsq.resize((size_t)ksum);
  p->tw64.resize(2 * (size_t)ksum);
  for (int ax = 0, off = 0; ax < 3; off += Ks[ax], ++ax) {
    moduli(order, Ks[ax], p->bsq.data() + off);
    for (int k = 0; k < Ks[ax]; ++k) {
      const double ang = 2.0 * pi * (double)k / (double)Ks[ax];
      p->tw64[2 * (off + k)] = std::cos(ang);
      p->tw64[2 * (off + k) + 1] = -std::sin(ang);
    }
  }
  p->tw32.resize(2 * (size_t)ksum);
  for (int i = 0; i < 2 * ksum; ++i) p->tw32[i] = (float)p->tw64[i];

  hipError_t e = spme::prepare_kernels(K1, K2, K3, order, precision);
  if (e == hipSuccess) e = hipMemsetAsync(p->ws + L.ctrl, 0, 64 * sizeof(unsigned), p->stream);
  // bucket and overflow counts start at zero; each step's convolution
  // clears them again for the next
  if (e == hipSuccess) e = hipMemsetAsync(p->ws + L.bcnt, 0, L.bcnt2 - L.bcnt, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(p->ws + L.ovf, 0, 4 * sizeof(unsigned), p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p->ws + L.bsq, p->bsq.data(), sizeof(double) * ksum,
                       hipMemcpyHostToDevice, p->stream);
  if (e == hipSuccess) {
    if (precision != PME_FP64)
      e = hipMemcpyAsync(p->ws + L.tw, p->tw32.data(), sizeof(float) * 2 * ksum,
                         hipMemcpyHostToDevice, p->stream);
    else
      e = hipMemcpyAsync(p->ws + L.tw, p->tw64.data(), sizeof(double) * 2 * ksum,
                         hipMemcpyHostToDevice, p->stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) {
    delete p;
    return PME_EDEVICE;
  }
  Args& a = p->cur;
  a.K1 = K1;
  a.K2 = K2;
  a.K3 = K3;
  a.order = order;
  a.precision = precision;
  a.frac_bits = frac_bits;
  a.beta = beta;
  a.coulomb = coulomb;
  a.ws = p->ws;
  a.lay = L;
  *out = p;
  return PME_OK;
}

int pme_destroy(pme_plan* p) {
  if (p == nullptr) return PME_EINVAL;
  for (hipEvent_t e : p->event_pool) (void)hipEventDestroy(e);
  delete p;
  return PME_OK;
}

int pme_set_stream(pme_plan* p, void* stream) {
  if (p == nullptr) return PME_EINVAL;
  p->stream = static_cast<hipStream_t>(stream);
  return PME_OK;
}

int pme_set_debug(pme_plan* p, int keep_charge_grid) {
  if (p == nullptr) return PME_EINVAL;
  p->keep_grid = keep_charge_grid ? 1 : 0;
  return PME_OK;
}

namespace {

// Reciprocal vectors of a general cell, rec[3a + c] = component c of a*_a
// with a*_a . a_b = delta_ab: the cross products of the other two box rows
// over V = a_1 . (a_2 x a_3), each operation one rounding (no contraction),
// in this order -- the same recipe as the fixed-point grid's reference, so
// that fractional coordinates agree bit for bit.  False for a degenerate
// cell.
bool box_recip(const double* box, double* rec, double* vol) {
#pragma clang fp contract(off)
  auto cross = [](const double* u, const double* v, double* w) {
    w[0] = u[1] * v[2] - u[2] * v[1];
    w[1] = u[2] * v[0] - u[0] * v[2];
    w[2] = u[0] * v[1] - u[1] * v[0];
  };
  double c[3];
  cross(box + 3, box + 6, c);
  const double V = box[0] * c[0] + box[1] * c[1] + box[2] * c[2];
  if (!(std::fabs(V) > 0.0) || !std::isfinite(V)) return false;
  cross(box + 3, box + 6, rec + 0);
  cross(box + 6, box + 0, rec + 3);
  cross(box + 0, box + 3, rec + 6);
  for (int i = 0; i < 9; ++i) rec[i] /= V;
  *vol = std::fabs(V);
  return true;
}

// Validate one step's inputs and fill the per-step fields of a.
int set_inputs(pme_plan* p, Args& a, const double* pos, const double* q, int N,
               const double box[9]) {
  if (p == nullptr || box == nullptr || N < 0 || N > p->max_atoms) return PME_EINVAL;
  if (N > 0 && (pos == nullptr || q == nullptr)) return PME_EINVAL;
  for (int i = 0; i < 9; ++i)
    if (!is_fin(box[i])) return PME_EINVAL;
  const bool diag = box[1] == 0.0 && box[2] == 0.0 && box[3] == 0.0 && box[5] == 0.0 &&
                    box[6] == 0.0 && box[7] == 0.0;
  if (diag && !(box[0] > 0.0 && box[4] > 0.0 && box[8] > 0.0)) return PME_EINVAL;
  double rec[9], vol = 0.0;
  if (!diag && !box_recip(box, rec, &vol)) return PME_EINVAL;
  a.N = N;
  a.n_chunks = (N + spme::kChunk - 1) / spme::kChunk;
  a.pos = pos;
  a.q = q;
  a.triclinic = diag ? 0 : 1;
  if (diag) {
    a.L[0] = box[0];
    a.L[1] = box[4];
    a.L[2] = box[8];
    for (int d = 0; d < 3; ++d) a.invL[d] = 1.0 / a.L[d];
    a.volume = a.L[0] * a.L[1] * a.L[2];
    for (int i = 0; i < 9; ++i) a.rec[i] = (i % 4 == 0) ? a.invL[i / 4] : 0.0;
  } else {
    for (int i = 0; i < 9; ++i) a.rec[i] = rec[i];
    for (int d = 0; d < 3; ++d) {
      a.invL[d] = rec[4 * d];  // unused for a general cell
      a.L[d] = 1.0 / rec[4 * d];
    }
    a.volume = vol;
  }
  a.keep_grid = p->keep_grid;
  a.forces = nullptr;
  a.ev = nullptr;
  a.reduce_ev = 0;
  return PME_OK;
}

}  // namespace

int pme_spread(pme_plan* p, const double* pos, const double* q, int N, const double box[9]) {
  if (p == nullptr) return PME_EINVAL;
  Args& a = p->cur;
  int rc = set_inputs(p, a, pos, q, N, box);
  if (rc != PME_OK) return rc;
  if (p->state == kSpread || p->state == kDirty) {
    // the previous binning's counts were never moved on by a convolution
    if (spme::launch_clear_counts(a, p->stream) != hipSuccess) return PME_EDEVICE;
  }
  p->state = kDirty;
  rc = timed(p, 0, [&](const spme::Timing& t) { return spme::launch_bin(a, p->stream, t); });
  if (rc == PME_OK)
    rc = timed(p, 1, [&](const spme::Timing& t) { return spme::launch_spread_x(a, p->stream, t); });
  if (rc != PME_OK) return rc;
  p->grid_kept = p->keep_grid;
  p->state = kSpread;
  return PME_OK;
}

namespace {

// The convolution writes one energy/virial row per column; the rows are
// summed either by the next launch of the step (fused = true) or by a
// one-workgroup kernel right away.
int solve_impl(pme_plan* p, double* ev, bool fused) {
  // exactly once per spread: the convolution transforms the spectrum in
  // place and moves the bucket counts on
  if (p->state != kSpread) return PME_ESTATE;
  Args& a = p->cur;
  a.ev = ev;
  a.reduce_ev = 0;
  int rc = timed(p, 2, [&](const spme::Timing& t) { return spme::launch_conv(a, p->stream, t); });
  if (rc != PME_OK) p->state = kDirty;
  if (rc != PME_OK) return rc;
  if (ev != nullptr) {
    if (fused)
      a.reduce_ev = 1;
    else
      rc = device_error(spme::launch_reduce_ev(a, p->stream));
  }
  if (rc != PME_OK) return rc;
  p->state = kSolved;
  return PME_OK;
}

int gather_impl(pme_plan* p, double* forces, int accumulate) {
  if (p->state != kSolved) return PME_ESTATE;
  Args& a = p->cur;
  if (a.N > 0 && forces == nullptr) return PME_EINVAL;
  a.forces = forces;
  a.accumulate = accumulate ? 1 : 0;
  int rc = timed(p, 3, [&](const spme::Timing& t) { return spme::launch_interp(a, p->stream, t); });
  a.reduce_ev = 0;
  if (rc == PME_OK && p->timing) p->timed_steps++;
  return rc;
}

}  // namespace

int pme_solve(pme_plan* p, double* ev) {
  if (p == nullptr) return PME_EINVAL;
  return solve_impl(p, ev, false);
}

int pme_gather(pme_plan* p, double* forces, int accumulate) {
  if (p == nullptr) return PME_EINVAL;
  return gather_impl(p, forces, accumulate);
}

int pme_step(pme_plan* p, const double* pos, const double* q, int N, const double box[9],
             double* forces, int accumulate, double* ev) {
  if (p == nullptr) return PME_EINVAL;
  if (N > 0 && forces == nullptr) return PME_EINVAL;
  int rc = pme_spread(p, pos, q, N, box);
  if (rc == PME_OK) rc = solve_impl(p, ev, true);
  if (rc == PME_OK) rc = gather_impl(p, forces, accumulate);
  return rc;
}

int pme_bind(pme_plan* p, const double* pos, const double* q, int N, const double box[9],
             double* forces, int accumulate, double* ev) {
  if (p == nullptr) return PME_EINVAL;
  if (N > 0 && forces == nullptr) return PME_EINVAL;
  Args b = p->cur;  // plan constants (grid, order, precision, tables, layout)
  int rc = set_inputs(p, b, pos, q, N, box);
  if (rc != PME_OK) return rc;
  b.forces = forces;
  b.accumulate = accumulate ? 1 : 0;
  b.ev = ev;
  b.reduce_ev = ev != nullptr ? 1 : 0;
  if (hipMemcpy(p->ws + p->lay.args, &b, sizeof(Args), hipMemcpyHostToDevice) != hipSuccess)
    return PME_EDEVICE;
  p->bound = b;
  p->is_bound = 1;
  return PME_OK;
}

int pme_batch_run(pme_plan* const* plans, int n, void* stream) {
  if (n < 0 || (n > 0 && plans == nullptr)) return PME_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (plans[i] == nullptr) return PME_EINVAL;
    if (!plans[i]->is_bound) return PME_ESTATE;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // groups of at most kMaxBatch plans sharing (precision, grid, order)
  std::vector<std::vector<int>> groups;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const Args &a = plans[x]->bound, &b = plans[y]->bound;
    if (a.precision != b.precision) return a.precision < b.precision;
    if (a.K1 != b.K1) return a.K1 < b.K1;
    if (a.K2 != b.K2) return a.K2 < b.K2;
    if (a.K3 != b.K3) return a.K3 < b.K3;
    return a.order < b.order;
  });
  for (int i : order) {
    const Args& a = plans[i]->bound;
    if (!groups.empty()) {
      const Args& g = plans[groups.back()[0]]->bound;
      if (g.precision == a.precision && g.K1 == a.K1 && g.K2 == a.K2 && g.K3 == a.K3 &&
          g.order == a.order &&
          (int)groups.back().size() < spme::kMaxBatch) {
        groups.back().push_back(i);
        continue;
      }
    }
    groups.push_back({i});
  }
  std::vector<spme::BatchArgs> bts(groups.size());
  std::vector<Args> reps(groups.size());
  for (size_t g = 0; g < groups.size(); ++g) {
    spme::BatchArgs& bt = bts[g];
    bt.n = (int)groups[g].size();
    Args rep = plans[groups[g][0]]->bound;  // sizes the grids: largest system of the group
    rep.reduce_ev = 0;
    for (int k = 0; k < bt.n; ++k) {
      const pme_plan* p = plans[groups[g][k]];
      bt.sys[k] = reinterpret_cast<const Args*>(p->ws + p->lay.args);
      rep.N = std::max(rep.N, p->bound.N);
      rep.n_chunks = std::max(rep.n_chunks, p->bound.n_chunks);
      rep.reduce_ev |= p->bound.reduce_ev;
    }
    reps[g] = rep;
  }
  // binning does not depend on the grid: one launch per precision (the
  // order above is sorted by precision first)
  std::vector<spme::BatchArgs> bin_bts;
  std::vector<Args> bin_reps;
  for (int i : order) {
    const Args& a = plans[i]->bound;
    if (bin_bts.empty() || bin_reps.back().precision != a.precision ||
        bin_bts.back().n == spme::kMaxBatch) {
      bin_bts.push_back(spme::BatchArgs{});
      bin_bts.back().n = 0;
      bin_reps.push_back(a);
    }
    spme::BatchArgs& bt = bin_bts.back();
    bt.sys[bt.n++] = reinterpret_cast<const Args*>(plans[i]->ws + plans[i]->lay.args);
    bin_reps.back().N = std::max(bin_reps.back().N, a.N);
    bin_reps.back().n_chunks = std::max(bin_reps.back().n_chunks, a.n_chunks);
  }
  const spme::Timing none;
  // plans whose last binning was not followed by a convolution
  for (int i = 0; i < n; ++i) {
    pme_plan* p = plans[i];
    if (p->state == kSpread || p->state == kDirty) {
      if (spme::launch_clear_counts(p->bound, s) != hipSuccess) return PME_EDEVICE;
    }
    p->state = kDirty;
  }
  // stage by stage over the groups, all on one stream
  for (size_t g = 0; g < bin_bts.size(); ++g)
    if (spme::launch_bin(bin_reps[g], s, none, &bin_bts[g]) != hipSuccess) return PME_EDEVICE;
  for (int stage = 1; stage < spme::kNumKernels; ++stage) {
    for (size_t g = 0; g < groups.size(); ++g) {
      const Args& a = reps[g];
      const spme::BatchArgs* bt = &bts[g];
      hipError_t e = hipSuccess;
      switch (stage) {
        case 1: e = spme::launch_spread_x(a, s, none, bt); break;
        case 2: e = spme::launch_conv(a, s, none, bt); break;
        default: e = spme::launch_interp(a, s, none, bt); break;
      }
      if (e != hipSuccess) return PME_EDEVICE;
    }
  }
  for (int i = 0; i < n; ++i) {
    pme_plan* p = plans[i];
    p->cur = p->bound;
    p->cur.reduce_ev = 0;
    p->grid_kept = p->bound.keep_grid;
    p->state = kSolved;
  }
  return PME_OK;
}

size_t pme_debug_grid_bytes(pme_plan* p, int which) {
  if (p == nullptr) return 0;
  const size_t n = (size_t)p->K1 * p->K2 * p->K3, kh = (size_t)p->K1 / 2 + 1;
  const size_t real = p->precision != PME_FP64 ? 4 : 8;
  const size_t spec_cpx =
      p->precision == PME_FP32_FIXED_HALF || p->precision == PME_FP32_FIXED_BF16 ? 4 : 2 * real;
  switch (which) {
    case 0: return n * 8;
    case 1: return (size_t)p->K2 * p->K3 * kh * spec_cpx;
    case 2: return n * real;
    default: return 0;
  }
}

int pme_debug_grid(pme_plan* p, int which, void* dst) {
  if (p == nullptr || dst == nullptr) return PME_EINVAL;
  const size_t bytes = pme_debug_grid_bytes(p, which);
  if (bytes == 0) return PME_EINVAL;
  const size_t K1 = p->K1;
  const size_t real = p->precision != PME_FP64 ? 4 : 8;
  hipError_t e;
  switch (which) {
    case 0:
      if (p->state < kSpread || !p->grid_kept) return PME_ESTATE;
      e = hipMemcpyAsync(dst, p->ws + p->lay.dbg, bytes, hipMemcpyDeviceToDevice, p->stream);
      break;
    case 1:
      if (p->state < kSpread) return PME_ESTATE;
      e = hipMemcpyAsync(dst, p->ws + p->lay.spec, bytes, hipMemcpyDeviceToDevice, p->stream);
      break;
    default: {
      if (p->state < kSolved) return PME_ESTATE;
      // the potential rows, from the spectrum the step left in the workspace
      Args a = p->cur;
      a.reduce_ev = 0;
      e = spme::launch_inv_x(a, p->stream);
      if (e != hipSuccess) break;
      e = hipMemcpy2DAsync(dst, K1 * real, p->ws + p->lay.phi + (p->order - 1) * real,
                           (size_t)p->lay.phi_pitch * real, K1 * real, (size_t)p->K2 * p->K3,
                           hipMemcpyDeviceToDevice, p->stream);
      break;
    }
  }
  return device_error(e);
}

int pme_check(pme_plan* p, unsigned* flags) {
  if (p == nullptr || flags == nullptr) return PME_EINVAL;
  unsigned f = 0;
  hipError_t e = hipMemcpyAsync(&f, p->ws + p->lay.ctrl, sizeof(unsigned), hipMemcpyDeviceToHost,
                                p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e == hipSuccess) e = spme::launch_clear_flags(p->cur, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return PME_EDEVICE;
  *flags = f;
  if (f & PME_FLAG_NONFINITE) return PME_ENONFINITE;
  if (f & PME_FLAG_OVERFLOW) return PME_EOVERFLOW;
  if (f & PME_FLAG_BUCKETS) return PME_ESTATE;
  return PME_OK;
}

int pme_kernel_timing(pme_plan* p, int enable) {
  if (p == nullptr) return PME_EINVAL;
  p->timing = enable ? 1 : 0;
  return PME_OK;
}

int pme_kernel_times(pme_plan* p, double* ms, int n, int* steps) {
  if (p == nullptr || (n > 0 && ms == nullptr)) return PME_EINVAL;
  if (hipStreamSynchronize(p->stream) != hipSuccess) return PME_EDEVICE;
  for (const TimedLaunch& t : p->pending) {
    float el = 0.0f;
    if (hipEventElapsedTime(&el, t.start, t.stop) != hipSuccess) return PME_EDEVICE;
    if (t.kernel < n) ms[t.kernel] += el;
  }
  p->pending.clear();
  p->event_next = 0;
  if (steps) *steps = p->timed_steps;
  p->timed_steps = 0;
  return PME_OK;
}

}  // extern "C"
