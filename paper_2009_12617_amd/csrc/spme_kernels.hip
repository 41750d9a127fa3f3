// Host-side part of the SPME kernels shared by every precision: workspace
// layout, the variants each plan shape supports, the small bookkeeping
// kernels, and dispatch to the per-precision launch tables (the kernels of
// each precision are compiled in spme_kern_<precision>.hip from the
// templates in spme_kernels.h).
#include "spme_kernels.h"

namespace spme {

// Sum of the energy/virial rows by one wavefront (pme_solve outside a step).
__global__ __launch_bounds__(64) void k_reduce_ev(Args a) { reduce_ev(a); }

// Clears the bucket and overflow counts of a step whose binning ran without
// its convolution (one workgroup).
__global__ void k_clear_counts(Args a) {
  unsigned* bcnt = reinterpret_cast<unsigned*>(a.ws + a.lay.bcnt);
  const int nbins = 2 * a.K3 * nq_of(a.K2, a.precision != PME_FP64);
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) bcnt[b] = 0u;
  if (threadIdx.x == 0) reinterpret_cast<unsigned*>(a.ws + a.lay.ovf)[0] = 0u;
}

__global__ void k_clear_flags(unsigned* ctrl) {
  if (threadIdx.x == 0) ctrl[0] = 0u;
}

// Plan initialisation (one workgroup): the per-axis squared B-spline moduli
// |b_a(m)|^2 = 1 / |sum_{k=0}^{p-2} M_p(k+1) exp(2 pi i m k / K_a)|^2 and the
// twiddles exp(-2 pi i k / K_a), both from FP64 sines and cosines of exact
// multiples of pi (the twiddles then rounded once to the plan's real type);
// sticky flags and atom counts cleared.  mp[k] = M_p(k + 1).
__global__ __launch_bounds__(1024) void k_init_plan(Args a, PlanInit in) {
  const int K[3] = {a.K1, a.K2, a.K3};
  const int ksum = a.K1 + a.K2 + a.K3;
  double* bsq = reinterpret_cast<double*>(a.ws + a.lay.bsq);
  for (int i = threadIdx.x; i < ksum; i += blockDim.x) {
    const int ax = i < K[0] ? 0 : i < K[0] + K[1] ? 1 : 2;
    const int Ka = K[ax], m = i - (ax == 0 ? 0 : ax == 1 ? K[0] : K[0] + K[1]);
    double re = 0.0, im = 0.0;
    for (int k = 0; k <= a.order - 2; ++k) {
      double sn, cs;
      sincospi(2.0 * (double)(((long)m * k) % Ka) / (double)Ka, &sn, &cs);
      re += in.mp[k] * cs;
      im += in.mp[k] * sn;
    }
    bsq[i] = 1.0 / (re * re + im * im);
    double sn, cs;
    sincospi(2.0 * (double)m / (double)Ka, &sn, &cs);
    if (a.precision == PME_FP64) {
      reinterpret_cast<double*>(a.ws + a.lay.tw)[2 * i] = cs;
      reinterpret_cast<double*>(a.ws + a.lay.tw)[2 * i + 1] = -sn;
    } else {
      reinterpret_cast<float*>(a.ws + a.lay.tw)[2 * i] = (float)cs;
      reinterpret_cast<float*>(a.ws + a.lay.tw)[2 * i + 1] = (float)-sn;
    }
  }
  unsigned* ctrl = reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl);
  for (int i = threadIdx.x; i < 64; i += blockDim.x) ctrl[i] = 0u;
  const int nbins = 2 * a.K3 * nq_of(a.K2, a.precision != PME_FP64);
  unsigned* bcnt = reinterpret_cast<unsigned*>(a.ws + a.lay.bcnt);
  unsigned* bcnt2 = reinterpret_cast<unsigned*>(a.ws + a.lay.bcnt2);
  for (int b = threadIdx.x; b < nbins; b += blockDim.x) {
    bcnt[b] = 0u;
    bcnt2[b] = 0u;
  }
  if (threadIdx.x < 4) reinterpret_cast<unsigned*>(a.ws + a.lay.ovf)[threadIdx.x] = 0u;
}

// Writes one system's arguments to the device copy batched launches read
// (stream-ordered, so batched runs enqueued earlier keep the old copy).
__global__ void k_store_args(Args a, Args* dst) {
  if (threadIdx.x == 0) *dst = a;
}

const PrecOps* prec_ops(int precision) {
  switch (precision) {
    case PME_FP32_FIXED: return &kOpsFixed;
    case PME_FP64: return &kOpsDouble;
    case PME_FP32_FIXED_HALF: return &kOpsHalf;
    case PME_FP32_FIXED_BF16: return &kOpsBf16;
    default: return nullptr;
  }
}

template <class F>
hipError_t with_prec(int prec, F&& f) {
  if (prec == PME_FP32_FIXED) return f(PFixed{});
  if (prec == PME_FP64) return f(PDouble{});
  if (prec == PME_FP32_FIXED_HALF) return f(PHalf{});
  if (prec == PME_FP32_FIXED_BF16) return f(PBf16{});
  return hipErrorInvalidValue;
}

bool grid_supported(int K1, int K2, int K3) {
  return with_grid(K1, K2, K3, [](auto) { return hipSuccess; }) == hipSuccess;
}

unsigned variants_for(int K1, int K2, int K3, int order, int precision) {
  const PrecOps* ops = prec_ops(precision);
  if (ops == nullptr || !grid_supported(K1, K2, K3) || (order != 4 && order != 6)) return 0u;
  return ops->variants(K1, K2, K3, order);
}

// Built-in choices (measured on MI355X): one workgroup per column wherever a
// column has fewer than 8192 points (each extra launch costs more than the
// LDS work it spreads out) -- the register-resident transforms where the
// pencils allow them (FP32, 32 or 64 points), else the LDS-resident ones --
// and the fused interpolation except for p >= 6 on grids with K2 K3 >= 16384
// (where redoing the inverse x transform per bin costs 6.8x the grid).
void default_variants(int K1, int K2, int K3, int order, int precision, int* conv_mode,
                      int* interp_mode) {
  const unsigned v = variants_for(K1, K2, K3, order, precision);
  const bool big = (long)K2 * K3 >= 8192;
  if (!big && (v & kVarConvReg))
    *conv_mode = kConvReg;
  else
    *conv_mode =
        ((big && (v & kVarConvSplit)) || !(v & kVarConvFused)) ? kConvSplit : kConvFused;
  const bool isplit = order >= 6 && (long)K2 * K3 >= 16384;
  *interp_mode = (isplit || !(v & kVarInterpFused)) ? kInterpSplit : kInterpFused;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Energy/virial rows of a convolution variant: one per wavefront of the
// workgroups that convolve a column, times the K1/2+1 columns.
int ev_rows_for(int K1, int K2, int K3, int precision, int conv_mode) {
  int w = 0;
  (void)with_prec(precision, [&](auto pt) {
    using P = decltype(pt);
    return with_grid(K1, K2, K3, [&](auto gc) {
      using G = decltype(gc);
      if constexpr (conv_split_ok<P, G>())
        if (conv_mode == kConvSplit) w = (G::K2 / pass_cy<G>()) * (kPassThreads / 64);
      if constexpr (conv_fused_ok<P, G>())
        if (conv_mode == kConvFused) w = conv_threads<P, G>() / 64;
      if constexpr (conv_reg_ok<P, G>())
        if (conv_mode == kConvReg) w = conv_reg_threads<G>() / 64;
      return hipSuccess;
    });
  });
  return w * (K1 / 2 + 1);
}

bool layout_for(int K1, int K2, int K3, int order, int max_atoms, int precision, Layout* lay) {
  if (!grid_supported(K1, K2, K3) || (order != 4 && order != 6) || max_atoms < 0) return false;
  if (precision != PME_FP32_FIXED && precision != PME_FP64 && precision != PME_FP32_FIXED_HALF &&
      precision != PME_FP32_FIXED_BF16)
    return false;
  const bool fx = precision != PME_FP64;
  const bool reduced = precision == PME_FP32_FIXED_HALF || precision == PME_FP32_FIXED_BF16;
  const size_t real = fx ? 4 : 8, cpx = 2 * real;
  const size_t spec_cpx = reduced ? 4 : cpx;
  const size_t kh = (size_t)K1 / 2 + 1, ksum = (size_t)K1 + K2 + K3;
  const size_t plane = (size_t)K2 * K3;  // (y, z) points
  const int nch = (max_atoms + kMinChunk - 1) / kMinChunk;
  const int nq = nq_of(K2, fx);
  const size_t nbins = 2 * (size_t)K3 * nq;
  const size_t rsz = fx ? sizeof(RecF) : sizeof(RecD);
  const unsigned var = variants_for(K1, K2, K3, order, precision);
  Layout L{};
  size_t o = 0;
  L.ctrl = o;      o = align256(o + 64 * sizeof(unsigned));
  L.bsq = o;       o = align256(o + ksum * sizeof(double));
  L.tw = o;        o = align256(o + ksum * cpx);
  L.bcnt = o;      o = align256(o + nbins * sizeof(unsigned));
  L.bcnt2 = o;     o = align256(o + nbins * sizeof(unsigned));
  L.ovf = o;       o = align256(o + 4 * sizeof(unsigned));
  L.absq = o;      o = align256(o + (size_t)nch * sizeof(double));
  L.cap = bucket_cap(K3, nq, max_atoms);
  L.rec = o;       o = align256(o + nbins * (size_t)L.cap * rsz);
  L.orec = o;      o = align256(o + (size_t)max_atoms * rsz);
  L.orec_max = max_atoms;
  L.spec = o;      o = align256(o + plane * kh * spec_cpx);
  L.mid = L.spec;
  if (reduced && (var & kVarConvSplit)) {
    L.mid = o;     o = align256(o + plane * kh * cpx);
  }
  L.phi_pitch = phi_pitch_of(K1, order);
  L.phi = o;       o = align256(o + plane * L.phi_pitch * real);
  L.partial_rows = std::max({ev_rows_for(K1, K2, K3, precision, kConvFused),
                             ev_rows_for(K1, K2, K3, precision, kConvSplit),
                             ev_rows_for(K1, K2, K3, precision, kConvReg)});
  L.partial = o;   o = align256(o + (size_t)L.partial_rows * 8 * sizeof(double));
  L.dbg = o;       o = align256(o + plane * K1 * 8);
  L.args = o;      o = align256(o + sizeof(Args));
  L.total = o;
  L.n_chunks_max = nch;
  *lay = L;
  return true;
}

hipError_t prepare_kernels(int K1, int K2, int K3, int order, int precision) {
  const PrecOps* ops = prec_ops(precision);
  return ops == nullptr ? hipErrorInvalidValue : ops->prepare(K1, K2, K3, order);
}

hipError_t launch_bin(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  const PrecOps* ops = prec_ops(a.precision);
  return ops == nullptr ? hipErrorInvalidValue : ops->bin(a, s, t, bt);
}
hipError_t launch_spread_x(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  const PrecOps* ops = prec_ops(a.precision);
  return ops == nullptr ? hipErrorInvalidValue : ops->spread_x(a, s, t, bt);
}
hipError_t launch_conv(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  const PrecOps* ops = prec_ops(a.precision);
  return ops == nullptr ? hipErrorInvalidValue : ops->conv(a, s, t, bt);
}
hipError_t launch_inv_x(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  const PrecOps* ops = prec_ops(a.precision);
  return ops == nullptr ? hipErrorInvalidValue : ops->inv_x(a, s, t, bt);
}
hipError_t launch_interp(const Args& a, hipStream_t s, const Timing& t, const BatchArgs* bt) {
  const PrecOps* ops = prec_ops(a.precision);
  return ops == nullptr ? hipErrorInvalidValue : ops->interp(a, s, t, bt);
}

hipError_t launch_reduce_ev(const Args& a, hipStream_t s) {
  k_reduce_ev<<<dim3(1), dim3(64), 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_clear_counts(const Args& a, hipStream_t s) {
  k_clear_counts<<<dim3(1), dim3(1024), 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_init_plan(const Args& a, const PlanInit& in, hipStream_t s) {
  k_init_plan<<<dim3(1), dim3(1024), 0, s>>>(a, in);
  return hipGetLastError();
}

hipError_t launch_store_args(const Args& a, Args* dst, hipStream_t s) {
  k_store_args<<<dim3(1), dim3(64), 0, s>>>(a, dst);
  return hipGetLastError();
}

hipError_t launch_clear_flags(const Args& a, hipStream_t s) {
  k_clear_flags<<<dim3(1), dim3(64), 0, s>>>(reinterpret_cast<unsigned*>(a.ws + a.lay.ctrl));
  return hipGetLastError();
}

}  // namespace spme

#ifdef SPME_TRACE
// Trace builds only: point the phase trace of every precision's kernels at a
// device buffer of 5 * 1024 * 16 uint64 (or NULL to stop tracing).
extern "C" int spme_trace_set(void* buf) {
  const spme::PrecOps* all[4] = {&spme::kOpsFixed, &spme::kOpsDouble, &spme::kOpsHalf,
                                 &spme::kOpsBf16};
  for (const spme::PrecOps* o : all)
    if (o->trace_set(buf) != hipSuccess) return 5;
  return 0;
}
#endif
