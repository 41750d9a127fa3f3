// C ABI of the SPME step: argument validation, workspace layout, plan tables
// and launch sequencing.  All device work is enqueued on the plan's stream;
// the library allocates no device memory.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <algorithm>
#include <array>
#include <map>
#include <mutex>
#include <set>
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
  // kernel variants (pme_tuning)
  int conv_mode = 0, interp_mode = 0, bin_chunk = 1024;
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

// Copies the plan's kernel variants into its launch arguments.
void apply_tuning(pme_plan* p, Args& a) {
  a.conv_mode = p->conv_mode;
  a.interp_mode = p->interp_mode;
  a.bin_chunk = p->bin_chunk;
  a.ev_rows = spme::ev_rows_for(p->K1, p->K2, p->K3, p->precision, p->conv_mode);
}

// Raises the dynamic-LDS limits of a (precision, grid, order)'s kernels once
// per process and device (hipFuncSetAttribute is a host call of its own per
// kernel; plans are created in serving loops).  A fixed table, so that the
// allocation-free step allocates no host memory either.
hipError_t prepare_kernels_once(int K1, int K2, int K3, int order, int precision) {
  static std::mutex mu;
  static std::array<std::array<int, 6>, 256> done;
  static int ndone = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  const std::array<int, 6> key{dev, K1, K2, K3, order, precision};
  std::lock_guard<std::mutex> lock(mu);
  for (int i = 0; i < ndone; ++i)
    if (done[i] == key) return hipSuccess;
  e = spme::prepare_kernels(K1, K2, K3, order, precision);
  if (e == hipSuccess && ndone < (int)done.size()) done[ndone++] = key;
  return e;
}

// Fills a plan for (grid, order, beta, max_atoms, precision, F, c) over
// `ws` and enqueues its initialisation launch on `stream`.  Arguments were
// validated by the caller.
int init_plan(pme_plan* p, int K1, int K2, int K3, int order, double beta, int max_atoms,
              int precision, int frac_bits, double coulomb, char* ws, size_t ws_bytes,
              hipStream_t stream, const Layout& L) {
  p->K1 = K1;
  p->K2 = K2;
  p->K3 = K3;
  p->order = order;
  p->precision = precision;
  p->frac_bits = frac_bits;
  p->max_atoms = max_atoms;
  p->beta = beta;
  p->coulomb = coulomb;
  p->ws = ws;
  p->ws_bytes = ws_bytes;
  p->stream = stream;
  p->lay = L;
  spme::default_variants(K1, K2, K3, order, precision, &p->conv_mode, &p->interp_mode);
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
  apply_tuning(p, a);
  // the plan tables are computed on the device from M_p at the integers
  spme::PlanInit init{};
  for (int k = 0; k <= order - 2; ++k) init.mp[k] = bspline_at(order, k + 1.0);
  hipError_t e = prepare_kernels_once(K1, K2, K3, order, precision);
  if (e == hipSuccess) e = spme::launch_init_plan(a, init, p->stream);
  return e == hipSuccess ? PME_OK : PME_EDEVICE;
}

// Argument checks shared by pme_create and the allocation-free step:
// PME_OK with *L filled, or the status to return.
int check_plan_args(int K1, int K2, int K3, int order, double beta, int max_atoms, int precision,
                    int* frac_bits, double* coulomb, Layout* L) {
  if (K1 < 2 || K2 < 2 || K3 < 2 || order < 3 || !(beta > 0.0) || !is_fin(beta) ||
      max_atoms < 0 ||
      (precision != PME_FP64 && precision != PME_FP32_FIXED && precision != PME_FP32_FIXED_HALF &&
       precision != PME_FP32_FIXED_BF16) ||
      !is_fin(*coulomb))
    return PME_EINVAL;
  if (*frac_bits == 0) *frac_bits = 32;
  if (*frac_bits < 16 || *frac_bits > 40) return PME_EINVAL;
  if (*coulomb == 0.0) *coulomb = 1.0;
  if (!spme::grid_supported(K1, K2, K3) || (order != 4 && order != 6) || max_atoms > kMaxAtoms)
    return PME_EUNSUPPORTED;
  if (!spme::layout_for(K1, K2, K3, order, max_atoms, precision, L)) return PME_EUNSUPPORTED;
  return PME_OK;
}

// PME_VAR_* bits a tuning needs.
unsigned variant_bits(const pme_tuning& t) {
  const unsigned c = t.conv == PME_CONV_FUSED ? PME_VAR_CONV_FUSED
                     : t.conv == PME_CONV_SPLIT ? PME_VAR_CONV_SPLIT
                                                : PME_VAR_CONV_REG;
  return c | (t.interp == PME_INTERP_FUSED ? PME_VAR_INTERP_FUSED : PME_VAR_INTERP_SPLIT);
}

}  // namespace

extern "C" {

int pme_version(void) { return 300; }

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
    case PME_EBUSY: return "no free batch slot or arena range";
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
  Layout L;
  const int rc = check_plan_args(K1, K2, K3, order, beta, max_atoms, precision, &frac_bits,
                                 &coulomb, &L);
  if (rc != PME_OK) return rc;
  if (workspace == nullptr || workspace_bytes < L.total ||
      (reinterpret_cast<uintptr_t>(workspace) & 255u) != 0)
    return PME_EWORKSPACE;
  pme_plan* p = new (std::nothrow) pme_plan();
  if (p == nullptr) return PME_EDEVICE;
  if (init_plan(p, K1, K2, K3, order, beta, max_atoms, precision, frac_bits, coulomb,
                static_cast<char*>(workspace), workspace_bytes, static_cast<hipStream_t>(stream),
                L) != PME_OK) {
    delete p;
    return PME_EDEVICE;
  }
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
  a.n_chunks = (N + p->bin_chunk - 1) / p->bin_chunk;
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
  apply_tuning(p, a);
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

int pme_step_probe(pme_plan* p, const double* pos, const double* q, int N, const double box[9],
                   double* forces, double* ev, int repeat) {
  if (p == nullptr) return PME_EINVAL;
  if (repeat < PME_PROBE_NONE || repeat > PME_PROBE_CLEAR) return PME_EINVAL;
  if (N > 0 && forces == nullptr) return PME_EINVAL;
  int rc = pme_spread(p, pos, q, N, box);
  if (rc == PME_OK && repeat == PME_PROBE_SPREAD)
    rc = device_error(spme::launch_spread_x(p->cur, p->stream));
  if (rc == PME_OK) rc = solve_impl(p, ev, true);
  if (rc == PME_OK) rc = gather_impl(p, forces, 0);
  if (rc != PME_OK) return rc;
  const Args& a = p->cur;
  switch (repeat) {
    case PME_PROBE_INTERP:
      // the same forces again (the energy rows were already summed)
      rc = device_error(spme::launch_interp(a, p->stream));
      break;
    case PME_PROBE_CONV:
      // on the spectrum the interpolation has used; the next spread rewrites
      // it, and the counts it moves on are already zero
      rc = device_error(spme::launch_conv(a, p->stream));
      p->state = kDirty;
      break;
    case PME_PROBE_BIN:
      // binning into the buckets the interpolation has used, its counts
      // cleared again for the next step
      rc = device_error(spme::launch_bin(a, p->stream));
      if (rc == PME_OK) rc = device_error(spme::launch_clear_counts(a, p->stream));
      break;
    case PME_PROBE_CLEAR:
      rc = device_error(spme::launch_clear_counts(a, p->stream));
      break;
    default:
      break;
  }
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
  if (spme::launch_store_args(b, reinterpret_cast<Args*>(p->ws + p->lay.args), p->stream) !=
      hipSuccess)
    return PME_EDEVICE;
  p->bound = b;
  p->is_bound = 1;
  return PME_OK;
}

}  // extern "C"

namespace {

// Plans that run together in one launch of each kernel: same precision,
// grid, order and variants.
bool same_group(const Args& a, const Args& b) {
  return a.precision == b.precision && a.K1 == b.K1 && a.K2 == b.K2 && a.K3 == b.K3 &&
         a.order == b.order && a.conv_mode == b.conv_mode && a.interp_mode == b.interp_mode &&
         a.bin_chunk == b.bin_chunk;
}

// Streams a batched run may fork its grid groups onto, with the events that
// fork them from and join them back into the calling stream.
struct Fork {
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> joined;  // one per fork stream
  hipEvent_t start = nullptr;
};

// One step of each bound plan.  Without fork streams: one binning launch per
// (precision, chunk), then spreading, convolution and interpolation once per
// grid group, every launch on s in stage order.  With them: each grid group
// runs its own binning, spreading, convolution and interpolation on a fork
// stream, the groups concurrently, joining s at the end.
int batch_run_impl(pme_plan* const* plans, int n, hipStream_t s, const Fork* fork) {
  if (n < 0 || (n > 0 && plans == nullptr)) return PME_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (plans[i] == nullptr) return PME_EINVAL;
    if (!plans[i]->is_bound) return PME_ESTATE;
  }
  {
    // a plan twice would bin its atoms twice into one set of buckets
    std::vector<const pme_plan*> seen(plans, plans + n);
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end()) return PME_EINVAL;
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
    const Args &a = plans[x]->bound, &b = plans[y]->bound;
    const std::array<int, 8> ka{a.precision, a.bin_chunk, a.K1, a.K2, a.K3, a.order, a.conv_mode,
                                a.interp_mode};
    const std::array<int, 8> kb{b.precision, b.bin_chunk, b.K1, b.K2, b.K3, b.order, b.conv_mode,
                                b.interp_mode};
    return ka < kb;
  });
  // groups of at most kMaxBatch plans (kernel launches)
  std::vector<std::vector<int>> groups;
  for (int i : order) {
    if (!groups.empty() && same_group(plans[groups.back()[0]]->bound, plans[i]->bound) &&
        (int)groups.back().size() < spme::kMaxBatch) {
      groups.back().push_back(i);
      continue;
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
  // binning does not depend on the grid: one launch per (precision, chunk)
  // (the order above is sorted by those first)
  std::vector<spme::BatchArgs> bin_bts;
  std::vector<Args> bin_reps;
  for (int i : order) {
    const Args& a = plans[i]->bound;
    if (bin_bts.empty() || bin_reps.back().precision != a.precision ||
        bin_reps.back().bin_chunk != a.bin_chunk || bin_bts.back().n == spme::kMaxBatch) {
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
  const int nfork = (fork != nullptr && groups.size() > 1)
                        ? (int)std::min(fork->streams.size(), groups.size())
                        : 0;
  if (nfork == 0) {
    for (size_t g = 0; g < bin_bts.size(); ++g)
      if (spme::launch_bin(bin_reps[g], s, none, &bin_bts[g]) != hipSuccess) return PME_EDEVICE;
    // stage by stage over the groups, all on one stream
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
  } else {
    // groups dealt to the fork streams, largest grids first (they take
    // longest), each stream running its groups' stages in order, binning
    // included (a group's chain then starts without waiting for the
    // binning of the others)
    if (hipEventRecord(fork->start, s) != hipSuccess) return PME_EDEVICE;
    for (int f = 0; f < nfork; ++f)
      if (hipStreamWaitEvent(fork->streams[f], fork->start, 0) != hipSuccess) return PME_EDEVICE;
    std::vector<size_t> by_size(groups.size());
    for (size_t g = 0; g < groups.size(); ++g) by_size[g] = g;
    std::stable_sort(by_size.begin(), by_size.end(), [&](size_t x, size_t y) {
      const long vx = (long)reps[x].K1 * reps[x].K2 * reps[x].K3 * bts[x].n;
      const long vy = (long)reps[y].K1 * reps[y].K2 * reps[y].K3 * bts[y].n;
      return vx > vy;
    });
    for (size_t k = 0; k < by_size.size(); ++k) {
      const size_t g = by_size[k];
      hipStream_t fs = fork->streams[k % nfork];
      const Args& a = reps[g];
      const spme::BatchArgs* bt = &bts[g];
      if (spme::launch_bin(a, fs, none, bt) != hipSuccess ||
          spme::launch_spread_x(a, fs, none, bt) != hipSuccess ||
          spme::launch_conv(a, fs, none, bt) != hipSuccess ||
          spme::launch_interp(a, fs, none, bt) != hipSuccess)
        return PME_EDEVICE;
    }
    for (int f = 0; f < nfork; ++f) {
      if (hipEventRecord(fork->joined[f], fork->streams[f]) != hipSuccess ||
          hipStreamWaitEvent(s, fork->joined[f], 0) != hipSuccess)
        return PME_EDEVICE;
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

}  // namespace

extern "C" {

int pme_batch_run(pme_plan* const* plans, int n, void* stream) {
  return batch_run_impl(plans, n, static_cast<hipStream_t>(stream), nullptr);
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
  p->pending.clear();
  p->event_next = 0;
  p->timed_steps = 0;
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


unsigned pme_tuning_variants(int K1, int K2, int K3, int order, int precision) {
  return spme::variants_for(K1, K2, K3, order, precision);
}

int pme_default_tuning(int K1, int K2, int K3, int order, int precision, pme_tuning* out) {
  if (out == nullptr) return PME_EINVAL;
  if (spme::variants_for(K1, K2, K3, order, precision) == 0u) return PME_EUNSUPPORTED;
  spme::default_variants(K1, K2, K3, order, precision, &out->conv, &out->interp);
  out->bin_chunk = 1024;
  return PME_OK;
}

int pme_get_tuning(pme_plan* p, pme_tuning* out) {
  if (p == nullptr || out == nullptr) return PME_EINVAL;
  out->conv = p->conv_mode;
  out->interp = p->interp_mode;
  out->bin_chunk = p->bin_chunk;
  return PME_OK;
}

int pme_set_tuning(pme_plan* p, const pme_tuning* t) {
  if (p == nullptr || t == nullptr) return PME_EINVAL;
  if (t->bin_chunk != 256 && t->bin_chunk != 512 && t->bin_chunk != 1024) return PME_EINVAL;
  if ((t->conv != PME_CONV_FUSED && t->conv != PME_CONV_SPLIT && t->conv != PME_CONV_REG) ||
      (t->interp != PME_INTERP_FUSED && t->interp != PME_INTERP_SPLIT))
    return PME_EINVAL;
  const unsigned v = spme::variants_for(p->K1, p->K2, p->K3, p->order, p->precision);
  const unsigned need = variant_bits(*t);
  if ((v & need) != need) return PME_EUNSUPPORTED;
  // the convolution of a spread step must match its spread (energy rows)
  if (p->state == kSpread) return PME_ESTATE;
  p->conv_mode = t->conv;
  p->interp_mode = t->interp;
  p->bin_chunk = t->bin_chunk;
  apply_tuning(p, p->cur);
  return PME_OK;
}

int pme_autotune(pme_plan* p, const double* pos, const double* q, int N, const double box[9],
                 double* forces, double* ev, int reps, pme_tuning* best, double* best_us,
                 double* times_us, int max_times) {
  if (p == nullptr || reps < 1 || (max_times > 0 && times_us == nullptr)) return PME_EINVAL;
  if (N > 0 && forces == nullptr) return PME_EINVAL;
  const unsigned v = spme::variants_for(p->K1, p->K2, p->K3, p->order, p->precision);
  const int convs[3] = {PME_CONV_FUSED, PME_CONV_SPLIT, PME_CONV_REG};
  const int interps[2] = {PME_INTERP_FUSED, PME_INTERP_SPLIT};
  const int chunks[3] = {256, 512, 1024};
  std::vector<pme_tuning> cand;
  std::vector<double> mean_us;
  for (int c : convs)
    for (int it : interps)
      for (int ch : chunks) cand.push_back(pme_tuning{c, it, ch});
  mean_us.assign(cand.size(), -1.0);
  pme_tuning keep;
  pme_get_tuning(p, &keep);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return PME_EDEVICE;
  }
  int rc = PME_OK;
  for (int round = 0; round < 3 && rc == PME_OK; ++round) {
    for (size_t k = 0; k < cand.size() && rc == PME_OK; ++k) {
      const pme_tuning& t = cand[k];
      const unsigned need = variant_bits(t);
      if ((v & need) != need) continue;
      if (p->state == kSpread) p->state = kDirty;  // (a failed step left counts behind)
      rc = pme_set_tuning(p, &t);
      for (int w = 0; w < 3 && rc == PME_OK; ++w)
        rc = pme_step(p, pos, q, N, box, forces, 0, ev);
      if (rc == PME_OK && hipEventRecord(e0, p->stream) != hipSuccess) rc = PME_EDEVICE;
      for (int r = 0; r < reps && rc == PME_OK; ++r) rc = pme_step(p, pos, q, N, box, forces, 0, ev);
      if (rc == PME_OK && hipEventRecord(e1, p->stream) != hipSuccess) rc = PME_EDEVICE;
      if (rc == PME_OK && hipEventSynchronize(e1) != hipSuccess) rc = PME_EDEVICE;
      float ms = 0.0f;
      if (rc == PME_OK && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = PME_EDEVICE;
      if (rc == PME_OK) {
        const double us = 1e3 * ms / reps;
        mean_us[k] = mean_us[k] < 0.0 ? us : std::min(mean_us[k], us);
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != PME_OK) {
    pme_set_tuning(p, &keep);
    return rc;
  }
  size_t kb = cand.size();
  for (size_t k = 0; k < cand.size(); ++k)
    if (mean_us[k] >= 0.0 && (kb == cand.size() || mean_us[k] < mean_us[kb])) kb = k;
  if (kb == cand.size()) return PME_EUNSUPPORTED;
  for (int k = 0; k < max_times && k < (int)cand.size(); ++k) times_us[k] = mean_us[k];
  rc = pme_set_tuning(p, &cand[kb]);
  if (rc == PME_OK) rc = pme_step(p, pos, q, N, box, forces, 0, ev);
  if (rc == PME_OK && hipStreamSynchronize(p->stream) != hipSuccess) rc = PME_EDEVICE;
  if (best) *best = cand[kb];
  if (best_us) *best_us = mean_us[kb];
  return rc;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batch admission: resident systems inside one caller-owned arena.
// ---------------------------------------------------------------------------
struct pme_batch {
  char* arena = nullptr;
  size_t arena_bytes = 0;
  hipStream_t stream = nullptr;
  std::map<size_t, size_t> free_ranges;  // offset -> bytes, disjoint, merged
  struct Slot {
    pme_plan* plan = nullptr;
    size_t off = 0, bytes = 0;
    double *pos = nullptr, *q = nullptr, *forces = nullptr, *ev = nullptr;
    bool owned_io = false;  // buffers carved from the slot's arena range
  };
  std::vector<Slot> slots;  // plan == nullptr: free
  Fork fork;
  size_t used = 0;
};

namespace {

constexpr int kForkStreams = 3;  // with the batch's own stream: four hardware queues per process

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Inputs and outputs carved from the arena: pos [n][3], q [n], forces [n][3],
// ev [7], each 256-byte aligned.
size_t io_bytes(int n) {
  const size_t m = (size_t)std::max(n, 0);
  return align_up(m * 24) + align_up(m * 8) + align_up(m * 24) + align_up(7 * 8);
}

// First fit over the free ranges; SIZE_MAX when nothing fits.
size_t arena_take(pme_batch* b, size_t bytes) {
  for (auto it = b->free_ranges.begin(); it != b->free_ranges.end(); ++it) {
    if (it->second >= bytes) {
      const size_t off = it->first, rest = it->second - bytes;
      b->free_ranges.erase(it);
      if (rest > 0) b->free_ranges[off + bytes] = rest;
      b->used += bytes;
      return off;
    }
  }
  return SIZE_MAX;
}

// Returns a range, merged with the free ranges on either side.
void arena_give(pme_batch* b, size_t off, size_t bytes) {
  b->used -= bytes;
  auto next = b->free_ranges.lower_bound(off);
  if (next != b->free_ranges.end() && off + bytes == next->first) {
    bytes += next->second;
    next = b->free_ranges.erase(next);
  }
  if (next != b->free_ranges.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += bytes;
      return;
    }
  }
  b->free_ranges[off] = bytes;
}

// The fork streams and events of a batch, created at its first admission
// (creating a batch touches no device).
bool fork_ready(pme_batch* b) {
  if (b->fork.start != nullptr) return true;
  hipEvent_t start = nullptr;
  if (hipEventCreateWithFlags(&start, hipEventDisableTiming) != hipSuccess) return false;
  for (int f = 0; f < kForkStreams; ++f) {
    hipStream_t fs = nullptr;
    hipEvent_t ev = nullptr;
    if (hipStreamCreateWithFlags(&fs, hipStreamNonBlocking) != hipSuccess) break;
    if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipStreamDestroy(fs);
      break;
    }
    b->fork.streams.push_back(fs);
    b->fork.joined.push_back(ev);
  }
  if ((int)b->fork.streams.size() < kForkStreams) {
    for (hipStream_t fs : b->fork.streams) (void)hipStreamDestroy(fs);
    for (hipEvent_t ev : b->fork.joined) (void)hipEventDestroy(ev);
    b->fork.streams.clear();
    b->fork.joined.clear();
    (void)hipEventDestroy(start);
    return false;
  }
  b->fork.start = start;
  return true;
}

}  // namespace

extern "C" {

size_t pme_batch_footprint(const pme_system_desc* s) {
  if (s == nullptr) return 0;
  const size_t ws =
      align_up(pme_workspace_bytes(s->K1, s->K2, s->K3, s->order, s->max_atoms, s->precision));
  if (ws == 0) return 0;
  return s->pos != nullptr ? ws : ws + io_bytes(s->max_atoms);
}

int pme_batch_create(pme_batch** out, int max_systems, void* arena, size_t arena_bytes,
                     void* stream) {
  if (out == nullptr) return PME_EINVAL;
  *out = nullptr;
  if (max_systems < 1 || max_systems > 4096) return PME_EINVAL;
  if (arena == nullptr || (reinterpret_cast<uintptr_t>(arena) & 255u) != 0 || arena_bytes < 256)
    return PME_EWORKSPACE;
  pme_batch* b = new (std::nothrow) pme_batch();
  if (b == nullptr) return PME_EDEVICE;
  b->arena = static_cast<char*>(arena);
  b->arena_bytes = arena_bytes & ~(size_t)255;
  b->stream = static_cast<hipStream_t>(stream);
  b->free_ranges[0] = b->arena_bytes;
  b->slots.resize((size_t)max_systems);
  *out = b;
  return PME_OK;
}

int pme_batch_destroy(pme_batch* b) {
  if (b == nullptr) return PME_EINVAL;
  for (auto& sl : b->slots)
    if (sl.plan != nullptr) pme_destroy(sl.plan);
  for (hipStream_t fs : b->fork.streams) (void)hipStreamDestroy(fs);
  for (hipEvent_t ev : b->fork.joined) (void)hipEventDestroy(ev);
  if (b->fork.start) (void)hipEventDestroy(b->fork.start);
  delete b;
  return PME_OK;
}

int pme_batch_admit(pme_batch* b, const pme_system_desc* s, int* slot) {
  if (b == nullptr || s == nullptr || slot == nullptr) return PME_EINVAL;
  *slot = -1;
  const size_t need = pme_batch_footprint(s);
  if (need == 0) {
    // an argument error or an unsupported shape, as pme_create reports it
    const bool bad = s->max_atoms < 0 || s->K1 < 2 || s->K2 < 2 || s->K3 < 2 || s->order < 3;
    return bad ? PME_EINVAL : PME_EUNSUPPORTED;
  }
  int free_slot = -1;
  for (size_t k = 0; k < b->slots.size(); ++k)
    if (b->slots[k].plan == nullptr) {
      free_slot = (int)k;
      break;
    }
  if (free_slot < 0) return PME_EBUSY;
  const size_t off = arena_take(b, need);
  if (off == SIZE_MAX) return PME_EBUSY;
  if (!fork_ready(b)) {
    arena_give(b, off, need);
    return PME_EDEVICE;
  }
  pme_batch::Slot sl;
  sl.off = off;
  sl.bytes = need;
  sl.owned_io = s->pos == nullptr;
  size_t ws_bytes = need;
  if (sl.owned_io) {
    if (s->q != nullptr || s->forces != nullptr || s->ev != nullptr) {
      arena_give(b, off, need);
      return PME_EINVAL;
    }
    const size_t m = (size_t)std::max(s->max_atoms, 0);
    ws_bytes = need - io_bytes(s->max_atoms);
    char* io = b->arena + off + ws_bytes;
    sl.pos = reinterpret_cast<double*>(io);
    sl.q = reinterpret_cast<double*>(io + align_up(m * 24));
    sl.forces = reinterpret_cast<double*>(io + align_up(m * 24) + align_up(m * 8));
    sl.ev = reinterpret_cast<double*>(io + align_up(m * 24) + align_up(m * 8) + align_up(m * 24));
  } else {
    sl.pos = const_cast<double*>(s->pos);
    sl.q = const_cast<double*>(s->q);
    sl.forces = s->forces;
    sl.ev = s->ev;
  }
  int rc = pme_create(&sl.plan, s->K1, s->K2, s->K3, s->order, s->beta, s->max_atoms,
                      s->precision, 0, 0.0, b->arena + off, ws_bytes, b->stream);
  if (rc == PME_OK && s->K1 != 64 && s->K1 != 128) {
    // In a batched launch the chip is full, so work counts more than
    // launches: the fused interpolation transforms p (R + p - 1) / R times
    // the grid's x rows (each tile those it reads), the split form each row
    // once.  Where the rows have no register transform (K1 other than 64
    // and 128) the split form is the batch's choice.
    pme_tuning t;
    if (pme_get_tuning(sl.plan, &t) == PME_OK && t.interp != PME_INTERP_SPLIT) {
      t.interp = PME_INTERP_SPLIT;
      rc = pme_set_tuning(sl.plan, &t);
      if (rc != PME_OK) pme_destroy(sl.plan);
    }
  }
  if (rc == PME_OK) {
    rc = pme_bind(sl.plan, sl.pos, sl.q, s->N, s->box, sl.forces, 0, sl.ev);
    if (rc != PME_OK) pme_destroy(sl.plan);
  }
  if (rc != PME_OK) {
    arena_give(b, off, need);
    return rc;
  }
  b->slots[(size_t)free_slot] = sl;
  *slot = free_slot;
  return PME_OK;
}

int pme_batch_update(pme_batch* b, int slot, const double* pos, const double* q, int N,
                     const double box[9], double* forces, double* ev) {
  pme_plan* p = pme_batch_plan(b, slot);
  if (p == nullptr) return PME_EINVAL;
  pme_batch::Slot& sl = b->slots[(size_t)slot];
  if (sl.owned_io) {
    // the carved buffers stay; only N and the box change
    if (pos != nullptr || q != nullptr || forces != nullptr || ev != nullptr) return PME_EINVAL;
    return pme_bind(p, sl.pos, sl.q, N, box, sl.forces, 0, sl.ev);
  }
  const int rc = pme_bind(p, pos, q, N, box, forces, 0, ev);
  if (rc == PME_OK) {
    sl.pos = const_cast<double*>(pos);
    sl.q = const_cast<double*>(q);
    sl.forces = forces;
    sl.ev = ev;
  }
  return rc;
}

int pme_batch_io(pme_batch* b, int slot, double** pos, double** q, double** forces, double** ev) {
  if (pme_batch_plan(b, slot) == nullptr) return PME_EINVAL;
  const pme_batch::Slot& sl = b->slots[(size_t)slot];
  if (pos) *pos = sl.pos;
  if (q) *q = sl.q;
  if (forces) *forces = sl.forces;
  if (ev) *ev = sl.ev;
  return PME_OK;
}

int pme_batch_retire(pme_batch* b, int slot) {
  pme_plan* p = pme_batch_plan(b, slot);
  if (p == nullptr) return PME_EINVAL;
  pme_batch::Slot& sl = b->slots[(size_t)slot];
  pme_destroy(p);
  // the range is reused only by launches enqueued later on the same stream
  arena_give(b, sl.off, sl.bytes);
  sl = pme_batch::Slot{};
  return PME_OK;
}

int pme_batch_launch(pme_batch* b, const int* slots, int n) {
  if (b == nullptr || (slots != nullptr && n < 0)) return PME_EINVAL;
  std::vector<pme_plan*> plans;
  if (slots == nullptr) {
    for (auto& sl : b->slots)
      if (sl.plan != nullptr) plans.push_back(sl.plan);
  } else {
    for (int k = 0; k < n; ++k) {
      pme_plan* p = pme_batch_plan(b, slots[k]);
      if (p == nullptr) return PME_EINVAL;
      plans.push_back(p);
    }
  }
  if (plans.empty()) return PME_OK;
  return batch_run_impl(plans.data(), (int)plans.size(), b->stream,
                        b->fork.start != nullptr ? &b->fork : nullptr);
}

int pme_batch_stats(pme_batch* b, int* admitted, size_t* bytes_used, size_t* largest_free) {
  if (b == nullptr) return PME_EINVAL;
  int n = 0;
  for (auto& sl : b->slots) n += sl.plan != nullptr ? 1 : 0;
  size_t lf = 0;
  for (auto& fr : b->free_ranges) lf = std::max(lf, fr.second);
  if (admitted) *admitted = n;
  if (bytes_used) *bytes_used = b->used;
  if (largest_free) *largest_free = lf;
  return PME_OK;
}

pme_plan* pme_batch_plan(pme_batch* b, int slot) {
  if (b == nullptr || slot < 0 || (size_t)slot >= b->slots.size()) return nullptr;
  return b->slots[(size_t)slot].plan;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free step: the library's own static device scratch stands in
// for the caller's workspace.
// ---------------------------------------------------------------------------
namespace {

constexpr size_t kScratchBytes = PME_SCRATCH_BYTES;
// One copy per device, held until the process ends.  In host code this name
// is only a stand-in for the symbol: its device address comes from
// hipGetSymbolAddress, once per device with that device current.
__device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices];

hipError_t scratch_on_current_device(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" int pme_step_noalloc(int K1, int K2, int K3, int order, double beta, int precision,
                                int frac_bits, double coulomb, const double* pos, const double* q,
                                int N, const double box[9], double* forces, int accumulate,
                                double* ev, void* stream) {
  Layout L;
  int rc = check_plan_args(K1, K2, K3, order, beta, N, precision, &frac_bits, &coulomb, &L);
  if (rc != PME_OK) return rc;
  if (L.total > kScratchBytes) return PME_EWORKSPACE;
  if (box == nullptr || (N > 0 && (pos == nullptr || q == nullptr || forces == nullptr)))
    return PME_EINVAL;
  char* ws = nullptr;
  if (scratch_on_current_device(&ws) != hipSuccess) return PME_EDEVICE;
  // a host plan on the stack (no heap), over this device's scratch; the
  // initialisation launch rewrites the tables and clears every counter the
  // step relies on, whatever an earlier call left there
  pme_plan p;
  rc = init_plan(&p, K1, K2, K3, order, beta, N, precision, frac_bits, coulomb, ws, kScratchBytes,
                 static_cast<hipStream_t>(stream), L);
  if (rc != PME_OK) return rc;
  return pme_step(&p, pos, q, N, box, forces, accumulate, ev);
}
