// Device-side building blocks of the SPME step on gfx950 (CDNA4):
//   * complex arithmetic and radix-2/3/4/8 DFT butterflies,
//   * an LDS-resident Stockham FFT in which one pencil is owned by a group
//     of T lanes of a single 64-wide wavefront,
//   * the single-precision cardinal B-spline recursion and fixed-point
//     quantisation used by the charge-spreading stage.
//
// The paper computes the 3D FFT as 1D transforms along each axis (§III.B)
// with a streaming FFT unit whose log N stages are laid out in hardware
// (§IV.A, Fig. 3).  Here each 1D transform is a short sequence of radix
// stages over a pencil held in LDS; the order of stages and the radices are
// chosen per length so that every stage splits evenly over the pencil's lanes.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spme {

template <typename T>
struct cplx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cplx<T> c_add(cplx<T> a, cplx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> c_sub(cplx<T> a, cplx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> c_mul(cplx<T> a, cplx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename T>
__device__ __forceinline__ cplx<T> c_mulc(cplx<T> a, cplx<T> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename T>
__device__ __forceinline__ cplx<T> c_conj(cplx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cplx<T> c_scale(cplx<T> a, T s) { return {a.x * s, a.y * s}; }
// s * i * a for s = +1 / -1
template <int S, typename T>
__device__ __forceinline__ cplx<T> c_muli(cplx<T> a) {
  return S > 0 ? cplx<T>{-a.y, a.x} : cplx<T>{a.y, -a.x};
}

// One DPP move of a double within the wavefront (each half moved with the
// same control); lanes without a source, or outside row_mask, read 0.0.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  const unsigned lo =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROW_MASK, 0xf, false);
  const unsigned hi =
      (unsigned)__builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROW_MASK, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Inclusive prefix sums of V doubles across the 16 lanes of each DPP row
// (row_shr 1, 2, 4, 8).
template <int V>
__device__ __forceinline__ void row_scan_add(double* v) {
#pragma unroll
  for (int c = 0; c < V; ++c) v[c] += dpp_f64<0x111, 0xf>(v[c]);
#pragma unroll
  for (int c = 0; c < V; ++c) v[c] += dpp_f64<0x112, 0xf>(v[c]);
#pragma unroll
  for (int c = 0; c < V; ++c) v[c] += dpp_f64<0x114, 0xf>(v[c]);
#pragma unroll
  for (int c = 0; c < V; ++c) v[c] += dpp_f64<0x118, 0xf>(v[c]);
}

// wave_sums: an inclusive DPP scan of V doubles over the wavefront (rows,
// then row_bcast 15 and 31); lane 63 ends with the wavefront's sums.
// block_sums: sums over the block in a fixed order -- wave_sums, then the
// wavefront sums in wavefront order by a row scan in wavefront 0.  Thread 15 ends with the block sums in v.  Every
// thread must call it (at most 16 wavefronts); wred needs 16 * 8 doubles; it
// synchronises once and the caller synchronises before reusing wred.
template <int V>
__device__ __forceinline__ void wave_sums(double* v) {
  row_scan_add<V>(v);
#pragma unroll
  for (int c = 0; c < V; ++c) v[c] += dpp_f64<0x142, 0xa>(v[c]);
#pragma unroll
  for (int c = 0; c < V; ++c) v[c] += dpp_f64<0x143, 0xc>(v[c]);
}

template <int V>
__device__ __forceinline__ void block_sums(double* v, double* wred) {
  wave_sums<V>(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 63) {
#pragma unroll
    for (int c = 0; c < V; ++c) wred[wave * 8 + c] = v[c];
  }
  __syncthreads();
  if (wave == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int c = 0; c < V; ++c) v[c] = lane < nw ? wred[lane * 8 + c] : 0.0;
    row_scan_add<V>(v);
  }
}

// Prevents the compiler from moving LDS accesses across this point.  The FFT
// stages below are wave-synchronous: all lanes of a pencil sit in one
// wavefront, whose LDS instructions execute in program order, so a stage can
// read every element it needs and then overwrite them in place.
__device__ __forceinline__ void lds_order() { __asm__ __volatile__("" ::: "memory"); }

// ---------------------------------------------------------------------------
// DFT butterflies: y_u = sum_r v_r exp(S 2 pi i u r / R), in place.
// ---------------------------------------------------------------------------
template <int R, int S, typename T>
struct Dft;

template <int S, typename T>
struct Dft<2, S, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  }
};

template <int S, typename T>
struct Dft<3, S, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    const T h = T(0.86602540378443864676);  // sqrt(3)/2
    cplx<T> t = c_add(v[1], v[2]);
    cplx<T> d = c_sub(v[1], v[2]);
    cplx<T> m = {v[0].x - T(0.5) * t.x, v[0].y - T(0.5) * t.y};
    cplx<T> id = c_scale(c_muli<S>(d), h);
    v[0] = c_add(v[0], t);
    v[1] = c_add(m, id);
    v[2] = c_sub(m, id);
  }
};

template <int S, typename T>
struct Dft<4, S, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> a0 = c_add(v[0], v[2]), a1 = c_sub(v[0], v[2]);
    cplx<T> b0 = c_add(v[1], v[3]), b1 = c_muli<S>(c_sub(v[1], v[3]));
    v[0] = c_add(a0, b0);
    v[2] = c_sub(a0, b0);
    v[1] = c_add(a1, b1);
    v[3] = c_sub(a1, b1);
  }
};

template <int S, typename T>
struct Dft<8, S, T> {
  static __device__ __forceinline__ void run(cplx<T>* v) {
    cplx<T> e[4] = {v[0], v[2], v[4], v[6]};
    cplx<T> o[4] = {v[1], v[3], v[5], v[7]};
    Dft<4, S, T>::run(e);
    Dft<4, S, T>::run(o);
    const T c = T(0.70710678118654752440);
    // W8^1 = c (1 + S i), W8^2 = S i, W8^3 = c (-1 + S i)
    cplx<T> w1 = {c * (o[1].x - S * o[1].y), c * (o[1].y + S * o[1].x)};
    cplx<T> w2 = c_muli<S>(o[2]);
    cplx<T> w3 = {c * (-o[3].x - S * o[3].y), c * (-o[3].y + S * o[3].x)};
    v[0] = c_add(e[0], o[0]);
    v[4] = c_sub(e[0], o[0]);
    v[1] = c_add(e[1], w1);
    v[5] = c_sub(e[1], w1);
    v[2] = c_add(e[2], w2);
    v[6] = c_sub(e[2], w2);
    v[3] = c_add(e[3], w3);
    v[7] = c_sub(e[3], w3);
  }
};

// ---------------------------------------------------------------------------
// Radix plans.  fft_lanes(N) lanes share one N-point pencil; every stage's
// butterfly count N/R is a multiple of it.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int fft_nstages(int N) {
  return N == 8 ? 2 : N == 12 ? 3 : N == 16 ? 2 : N == 18 ? 3 : N == 24 ? 3 : N == 32 ? 2
       : N == 36 ? 4 : N == 48 ? 3 : N == 64 ? 2 : N == 72 ? 5 : N == 96 ? 4 : N == 128 ? 3 : 0;
}
__host__ __device__ constexpr int fft_radix(int N, int s) {
  return N == 8 ? (s == 0 ? 4 : 2)
       : N == 12 ? (s < 2 ? 2 : 3)
       : N == 16 ? 4
       : N == 18 ? (s == 0 ? 2 : 3)
       : N == 24 ? (s == 0 ? 4 : s == 1 ? 2 : 3)
       : N == 32 ? (s == 0 ? 8 : 4)
       : N == 36 ? (s < 2 ? 2 : 3)
       : N == 48 ? (s < 2 ? 4 : 3)
       : N == 64 ? 8
       : N == 72 ? (s < 3 ? 2 : 3)
       : N == 96 ? (s < 2 ? 4 : s == 2 ? 2 : 3)
       : N == 128 ? (s == 0 ? 8 : 4)
       : 0;
}
// (a power of two that divides every stage's butterfly count: 18 has stages
// of 9 and 6 butterflies, so one lane per pencil)
__host__ __device__ constexpr int fft_lanes(int N) {
  return N == 8 ? 2 : N == 12 ? 2 : N == 16 ? 4 : N == 18 ? 1 : N == 24 ? 2 : N == 32 ? 4
       : N == 36 ? 2 : N == 48 ? 4 : N == 64 ? 8 : N == 72 ? 4 : N == 96 ? 8 : N == 128 ? 16 : 0;
}
__host__ __device__ constexpr int fft_span(int N, int s) {  // product of the radices before s
  return s == 0 ? 1 : fft_span(N, s - 1) * fft_radix(N, s - 1);
}
__host__ __device__ constexpr bool fft_supported(int N) { return fft_nstages(N) > 0; }

// One Stockham stage: butterfly b reads x[b + r N/R], multiplies by
// W_{Ls R}^{(b mod Ls) r}, applies the radix-R DFT and writes output u to
// (b / Ls) Ls R + (b mod Ls) + u Ls.  Twiddles come from a table
// tw[k] = exp(-2 pi i k / (N twstep)), k < N twstep.
template <typename T, int N, int R, int LS, int S>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int stride, int lane,
                                          const cplx<T>* tw, int twstep) {
  constexpr int NT = fft_lanes(N);
  constexpr int NB = N / R;
  constexpr int BPL = NB / NT;
  static_assert(NB % NT == 0, "radix plan does not split over the pencil's lanes");
  cplx<T> v[BPL][R];
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    const int b = lane + i * NT;
#pragma unroll
    for (int r = 0; r < R; ++r) v[i][r] = buf[(b + r * NB) * stride];
  }
  lds_order();
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    const int b = lane + i * NT;
    const int j = b % LS;
    if (LS > 1) {
#pragma unroll
      for (int r = 1; r < R; ++r) {
        const cplx<T> w = tw[j * r * (N / (LS * R)) * twstep];
        v[i][r] = S < 0 ? c_mul(v[i][r], w) : c_mulc(v[i][r], w);
      }
    }
    Dft<R, S, T>::run(v[i]);
  }
#pragma unroll
  for (int i = 0; i < BPL; ++i) {
    const int b = lane + i * NT;
    const int j = b % LS, k = b / LS;
#pragma unroll
    for (int u = 0; u < R; ++u) buf[(k * LS * R + j + u * LS) * stride] = v[i][u];
  }
  lds_order();
}

template <typename T, int N, int S, int STAGE, bool DONE = (STAGE >= fft_nstages(N))>
struct StockhamRun {
  static __device__ __forceinline__ void run(cplx<T>* buf, int stride, int lane,
                                             const cplx<T>* tw, int twstep) {
    fft_stage<T, N, fft_radix(N, STAGE), fft_span(N, STAGE), S>(buf, stride, lane, tw, twstep);
    StockhamRun<T, N, S, STAGE + 1>::run(buf, stride, lane, tw, twstep);
  }
};
template <typename T, int N, int S, int STAGE>
struct StockhamRun<T, N, S, STAGE, true> {
  static __device__ __forceinline__ void run(cplx<T>*, int, int, const cplx<T>*, int) {}
};

// In-place unnormalised N-point DFT with exp(S 2 pi i jk/N) of the pencil
// buf[k*stride], k < N, by lane `lane` (0..fft_lanes(N)-1) of its group.
template <typename T, int N, int S>
__device__ __forceinline__ void fft_pencil(cplx<T>* buf, int stride, int lane,
                                           const cplx<T>* tw, int twstep) {
  static_assert(fft_supported(N), "unsupported FFT length");
  StockhamRun<T, N, S, 0>::run(buf, stride, lane, tw, twstep);
}

// ---------------------------------------------------------------------------
// Real-to-complex along a row of N = 2M reals stored as M packed complex
// values z_n = x_{2n} + i x_{2n+1}: after the M-point forward FFT Z, the half
// spectrum is X_k = E_k + W_N^k O_k with E_k = (Z_k + conj Z_{M-k})/2 and
// O_k = (Z_k - conj Z_{M-k})/(2i), k = 0..M (W_N^M = -1).  Each lane handles
// the pairs (k, M-k) for k = lane, lane + NT, ... <= M/2.
// ---------------------------------------------------------------------------
template <typename T, int N, class Sink>
__device__ __forceinline__ void r2c_post(const cplx<T>* row, int lane, const cplx<T>* twN,
                                         Sink&& sink) {
  constexpr int M = N / 2;
  constexpr int NT = fft_lanes(M);
  constexpr int NP = M / 2 + 1;
  constexpr int PPL = (NP + NT - 1) / NT;
  cplx<T> za[PPL], zb[PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int k = lane + i * NT;
    if (k < NP) {
      za[i] = row[k];
      zb[i] = row[(M - k) % M];
    }
  }
  lds_order();
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int k = lane + i * NT;
    if (k < NP) {
      // X_k from (Z_k, Z_{M-k}); X_{M-k} from (Z_{M-k}, Z_k)
      const cplx<T> zk = za[i], zm = zb[i];
      cplx<T> e = c_scale(c_add(zk, c_conj(zm)), T(0.5));
      cplx<T> d = c_sub(zk, c_conj(zm));
      cplx<T> o = {T(0.5) * d.y, T(-0.5) * d.x};  // d / (2i)
      if (k == 0) {
        sink(0, c_add(e, o));
        sink(M, c_sub(e, o));
      } else {
        sink(k, c_add(e, c_mul(twN[k], o)));
        if (k != M - k) {
          cplx<T> e2 = c_scale(c_add(zm, c_conj(zk)), T(0.5));
          cplx<T> d2 = c_sub(zm, c_conj(zk));
          cplx<T> o2 = {T(0.5) * d2.y, T(-0.5) * d2.x};
          sink(M - k, c_add(e2, c_mul(twN[M - k], o2)));
        }
      }
    }
  }
}
// ... in place: X_0 .. X_M into the row.
template <typename T, int N>
__device__ __forceinline__ void r2c_post(cplx<T>* row, int lane, const cplx<T>* twN) {
  r2c_post<T, N>(row, lane, twN, [&](int k, const cplx<T>& x) { row[k] = x; });
  lds_order();
}

// Complex-to-real preparation: from the half spectrum X_0..X_M of a real
// row (N = 2M) build Y_k = A_k + i B_k, k < M, with A_k = X_k + conj X_{M-k}
// and B_k = (X_k - conj X_{M-k}) exp(+2 pi i k/N); the M-point inverse FFT of
// Y then holds x_{2n} + i x_{2n+1} (unnormalised).  Im X_0 and Im X_M are
// exactly zero for a real row and are dropped.
template <typename T, int N>
__device__ __forceinline__ void c2r_pre(cplx<T>* row, int lane, const cplx<T>* twN) {
  constexpr int M = N / 2;
  constexpr int NT = fft_lanes(M);
  constexpr int NP = M / 2 + 1;
  constexpr int PPL = (NP + NT - 1) / NT;
  cplx<T> xa[PPL], xb[PPL];
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int k = lane + i * NT;
    if (k < NP) {
      xa[i] = row[k];
      xb[i] = row[M - k];
    }
  }
  lds_order();
#pragma unroll
  for (int i = 0; i < PPL; ++i) {
    const int k = lane + i * NT;
    if (k < NP) {
      cplx<T> xk = xa[i], xm = xb[i];
      if (k == 0) {
        xk.y = T(0);
        xm.y = T(0);
      }
      cplx<T> a = c_add(xk, c_conj(xm));
      cplx<T> b = c_mulc(c_sub(xk, c_conj(xm)), twN[k]);
      row[k] = {a.x - b.y, a.y + b.x};  // A + i B
      if (k != 0 && k != M - k) {
        cplx<T> a2 = c_add(xm, c_conj(xk));
        cplx<T> b2 = c_mulc(c_sub(xm, c_conj(xk)), twN[M - k]);
        row[M - k] = {a2.x - b2.y, a2.y + b2.x};
      }
    }
  }
  lds_order();
}

// ---------------------------------------------------------------------------
// Cardinal B-splines.  For an atom at grid coordinate g + w the p weights of
// points g-p+1+j are theta_j = M_p(w + p-1-j), built by the order recursion
// d_n[j] = ((w + n-1-j) d_{n-1}[j-1] + (j+1-w) d_{n-1}[j]) / (n-1) from
// d_2 = {1-w, w}; derivatives from the order p-1 array,
// dtheta_j = d_{p-1}[j-1] - d_{p-1}[j].  In single precision the operation
// sequence is fixed (no contraction, 1/(n-1) as a rounded constant) because
// the fixed-point grid must reproduce bit for bit.
// ---------------------------------------------------------------------------
template <int P, typename T>
__device__ __forceinline__ void bspline(T w, T* th, T* dth) {
#pragma clang fp contract(off)
  T d[P];
  d[0] = T(1) - w;
  d[1] = w;
#pragma unroll
  for (int n = 3; n <= P; ++n) {
    if (n == P && dth != nullptr) {
#pragma unroll
      for (int j = 0; j < P; ++j) {
        const T lo = (j >= 1) ? d[j - 1] : T(0);
        const T hi = (j <= P - 2) ? d[j] : T(0);
        dth[j] = lo - hi;
      }
    }
    const T c = T(1) / T(n - 1);
    T e[P];
#pragma unroll
    for (int j = 0; j < n; ++j) {
      const T t1 = (j >= 1) ? (w + T(n - 1 - j)) * d[j - 1] : T(0);
      const T t2 = (j <= n - 2) ? (T(j + 1) - w) * d[j] : T(0);
      e[j] = (t1 + t2) * c;
    }
#pragma unroll
    for (int j = 0; j < n; ++j) d[j] = e[j];
  }
#pragma unroll
  for (int j = 0; j < P; ++j) th[j] = d[j];
}

// Grid coordinate along one axis (orthorhombic cell): s = x / L through the
// host-rounded 1/L, wrapped into [0,1), u = K s, g = floor(u) mod K and
// w = u - floor(u), all in FP64 without contraction.  Returns false for a
// non-finite coordinate.
__device__ __forceinline__ bool grid_coord(double x, double invL, int K, int* g, double* w);

// Fractional coordinate along a*_a of a general cell: the dot product
// r . a*_a in the order (r_0 a_0 + r_1 a_1) + r_2 a_2, one rounding per
// operation.
__device__ __forceinline__ double frac_general(const double* r, const double* astar) {
#pragma clang fp contract(off)
  return (r[0] * astar[0] + r[1] * astar[1]) + r[2] * astar[2];
}

// Base grid index and offset from a fractional coordinate s (any real).
__device__ __forceinline__ bool grid_coord_s(double s, int K, int* g, double* w) {
#pragma clang fp contract(off)
  s = s - floor(s);                        // NaN for a non-finite x
  const bool ok = (s >= 0.0) && (s <= 1.0);
  if (!ok) s = 0.0;
  const double u = s * (double)K;
  const double fl = floor(u);              // 0 <= fl <= K
  int gi = (int)fl;
  if (gi >= K) gi -= K;                    // s rounded up to 1: u == K, w == 0
  *g = gi;
  *w = u - fl;
  return ok;
}

// Diagonal box: s = x (1/L) in one rounding.
__device__ __forceinline__ bool grid_coord(double x, double invL, int K, int* g, double* w) {
#pragma clang fp contract(off)
  return grid_coord_s(x * invL, K, g, w);
}

// 64-bit fixed-point contribution: round-half-even of c 2^F.  c 2^F is exact
// in FP64; adding 1.5 2^52 in one fused operation rounds it to an integer in
// the default round-to-nearest-even mode, and the integer is the difference
// of the two bit patterns (valid for |c 2^F| < 2^51, which the plan's
// headroom check guarantees).
__device__ __forceinline__ long long to_fixed(float c, double scale) {
  const double magic = 6755399441055744.0;  // 1.5 * 2^52
  const double d = __fma_rn((double)c, scale, magic);
  return __double_as_longlong(d) - __double_as_longlong(magic);
}

}  // namespace spme
