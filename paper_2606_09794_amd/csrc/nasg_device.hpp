// Device-side building blocks of the NASGabor / SH-3 evaluators (gfx950).
//
// - storage decode for float32 / bfloat16 lobe parameters, and the
//   nontemporal (streaming) accesses for data used once,
// - reductions over the `P` consecutive lanes that share a primitive, done
//   with DPP row operations (no LDS, no atomics, fixed order),
// - the per-lobe normaliser (Section 5.1) and its log-derivatives, in FP64
//   and, for the range of lam and lam (1 + a) where nothing cancels badly,
//   in FP32.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nasg {

constexpr double kPi = 3.141592653589793238462643383279502884;
constexpr double kInvTwoPi = 0.159154943091895335768883763372514362;
constexpr double kInvPi = 0.318309886183790671537767526745028724;

// ---------------------------------------------------------------- storage
// Data that a launch touches once is accessed nontemporally: the streaming
// cache policy keeps it from displacing what is still to be reused (the
// cameras, the log table). The appearance kernels do so in their streaming
// flavour (ONCE), used where it is safe and pays: one lane per primitive, so
// that a wave's access covers whole cache lines (with P lanes a wave covers
// part of a line, e.g. 4 x 64/P bytes of a colour-weight row, its neighbour
// the rest, and a streamed line can be gone before the second part is read
// or be written out twice), and a launch that reads every lobe record and
// writes every output once (all views in one chunk, no accumulation onto
// earlier results; otherwise later chunks, or the accumulating caller's next
// launch, read the same data again and it should stay cached).
typedef float f32x4_nt __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_nt __attribute__((ext_vector_type(2)));

template <class T>
__device__ inline T load_once(const T* p) {
  return __builtin_nontemporal_load(p);
}
template <class T>
__device__ inline void store_once(T v, T* p) {
  __builtin_nontemporal_store(v, p);
}
template <bool NT, class T>
__device__ inline T load_if(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  return *p;
}
template <bool NT, class T>
__device__ inline void store_if(T v, T* p) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v, p);
  } else {
    *p = v;
  }
}

template <bool BF16>
struct Store;

template <>
struct Store<false> {
  template <bool ONCE>
  __device__ static inline float4 load4(const void* p, int64_t idx) {
    const f32x4_nt v = load_if<ONCE>(reinterpret_cast<const f32x4_nt*>(p) + idx);
    return make_float4(v.x, v.y, v.z, v.w);
  }
  template <bool ONCE>
  __device__ static inline float load1(const void* p, int64_t idx) {
    return load_if<ONCE>(reinterpret_cast<const float*>(p) + idx);
  }
};

template <>
struct Store<true> {
  // four bfloat16 values packed little-endian in 8 bytes
  template <bool ONCE>
  __device__ static inline float4 load4(const void* p, int64_t idx) {
    const u32x2_nt u = load_if<ONCE>(reinterpret_cast<const u32x2_nt*>(p) + idx);
    return make_float4(__uint_as_float(u.x << 16), __uint_as_float(u.x & 0xffff0000u),
                       __uint_as_float(u.y << 16), __uint_as_float(u.y & 0xffff0000u));
  }
  template <bool ONCE>
  __device__ static inline float load1(const void* p, int64_t idx) {
    const uint16_t u = load_if<ONCE>(reinterpret_cast<const uint16_t*>(p) + idx);
    return __uint_as_float(static_cast<uint32_t>(u) << 16);
  }
};

// ---------------------------------------------------------- lane-group sums
// All-reduce over aligned groups of P consecutive lanes (P <= 16, one DPP row).
// Call only where every lane of the wavefront is active: DPP reads an
// inactive lane as zero.
// quad_perm [1,0,3,2] and [2,3,0,1] give the quad sum; row_half_mirror pairs
// the two quads of a half-row; row_mirror pairs the two half-rows.

// The neighbour's value through a DPP move with zero fill (bound_ctrl), the
// form the compiler folds into the consuming add (v_add_f32_dpp).
template <int CTRL>
__device__ inline float dpp_f(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, true));
}

template <int P>
__device__ inline float group_sum(float x) {
  static_assert(P == 1 || P == 2 || P == 4 || P == 8 || P == 16, "lanes per primitive");
  if constexpr (P >= 2) x += dpp_f<0xB1>(x);
  if constexpr (P >= 4) x += dpp_f<0x4E>(x);
  if constexpr (P >= 8) x += dpp_f<0x141>(x);
  if constexpr (P >= 16) x += dpp_f<0x140>(x);
  return x;
}

// ------------------------------------------------- FP64 envelope helpers
// The envelope exponent X = ln(p E) reaches |X| ~ 1e2 where G still matters,
// and exp amplifies an absolute error of X into a relative error of G, so X
// is formed in FP64. The helpers below are purpose-built for that: a few FP64
// fused multiply-adds each (FP64 FMA issues at the non-packed FP32 rate on
// CDNA4), relative error ~1e-13, inputs restricted to the ranges that occur.

// a * b + c as a three-address v_fma_f64. Used in the once-per-lobe code,
// where the compiler otherwise picks the two-address form with a hoisted
// coefficient as the accumulator and copies it before every step.
__device__ __forceinline__ double fma3(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}

constexpr double kLn2Hi = 0.693145751953125;               // 2^-11 multiple
constexpr double kLn2Lo = 1.4286068203094172321214581765680755e-06;
constexpr double kLog2e = 1.442695040888963407359924681001892137;

// 1/x for x > 0 normal: the hardware estimate (relative error < 5e-8
// measured on gfx950) plus one Newton step (error ~ its square, ~2e-15).
__device__ inline double rcp64(double x) {
  const double y = __builtin_amdgcn_rcp(x);
  return fma(y, fma(-x, y, 1.0), y);
}

// 1/sqrt(x) and sqrt(x) for x > 0 normal: the hardware estimate and one
// Newton step, y1 = y + y (1 - x y^2)/2 (relative error ~ 1.5 times the
// square of the estimate's).
__device__ inline double rsqrt64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
__device__ inline double sqrt64(double x) { return x * rsqrt64(x); }

// ---------------------------------------- envelope helpers (per lobe-view)
// Where G is above the FP32 range floor, |X| <= ~1e2. A relative error eps of
// ln kappa or of e^B then moves X by at most ~2e2 eps (the derivative of X
// with respect to ln kappa is about X / ln kappa, and e^B - 1 enters as
// 2 lam (e^B - 1) with lam (1 - e^B) <= ~50), so eps ~ 1e-10 keeps G
// relatively accurate to ~1e-8. Near kappa = 1, where that derivative grows
// to 2 lam (1 + tau) ~ 2e6, ln kappa keeps an absolute error ~1e-16.

constexpr double kLn2 = 0.693147180559945309417232121458176568;

// One bucket of the ln table: 1/c (rounded) and -ln of that rounded value.
struct alignas(16) LogEntry {
  double inv_c;
  double ln_c;
};
constexpr int kLogBits = 7;
constexpr int kLogEntries = 1 << kLogBits;

// ln kappa for kappa in (0, 1), from a 128-entry table in LDS. kappa = m 2^e
// with m in [1/2, 1); the top seven mantissa bits of m select c (the bucket
// centre; c = 1 for the top bucket); r = m/c - 1 in one rounding, less
// `dkap`, the known rounding error of kappa itself (kappa as computed minus
// its exact value; it matters only in the top bucket, where r = kappa - 1);
// |r| <= 1/256 and ln kappa = e ln2 + ln c + ln(1 + r) with ln(1 + r) summed
// to r^4 (truncation |r|^5/5 <= 1.8e-13; relative r^4/5 in the top bucket,
// so ln kappa stays relatively accurate however close kappa is to 1).
__device__ inline int log_bucket(double m) {
  return (__double2hiint(m) >> (20 - kLogBits)) & (kLogEntries - 1);
}
// A constant held in a vector register the compiler cannot see through, so
// that a polynomial step with two constant operands (a coefficient times the
// variable plus a coefficient) still encodes as one fused multiply-add: the
// hardware takes at most one scalar operand besides literals, and without it
// the compiler copies the second constant into a register before every use.
__device__ __forceinline__ double vreg_const(double c) {
  double r;
  asm volatile("v_mov_b64 %0, %1" : "=v"(r) : "s"(c));
  return r;
}

// a * b + c with b a scalar operand (the one the encoding allows besides
// vector registers), so that no copy of c is made.
__device__ __forceinline__ double fma_vsv(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "s"(b), "v"(c));
  return d;
}

__device__ inline double log_finish(double m, int e, const LogEntry& t, double dkap,
                                    double third = 1.0 / 3.0) {
  const double r = fma(m, t.inv_c, -1.0) - dkap;
  double p = fma_vsv(r, -0.25, third);
  p = fma(p, r, -0.5);
  const double lp = fma(p, r * r, r);
  return fma(static_cast<double>(e), kLn2, t.ln_c + lp);
}
__device__ inline double log_kappa(double kap, double dkap, const LogEntry* tab) {
  int e;
  const double m = frexp(kap, &e);
  return log_finish(m, e, tab[log_bucket(m)], dkap);
}

// e^B and e^B - 1 for B <= 0 on the envelope path: B = n ln2 + r in one FMA
// (the rounding of ln2 costs |n| 2e-17, negligible wherever e^B matters),
// e^r - 1 = r q(r) with q the Taylor series of (e^r - 1)/r to r^7/8!
// (relative truncation r^8/9! <= 6e-10 at |r| = ln2/2, far smaller near
// B = 0 where 2 lam (e^B - 1) is large). e^B - 1 is formed as e^B - 1, an
// absolute error ~1e-16. B below -1e6 is clamped (e^B is 0 there).
__device__ inline void env_exp(double B, double& eb, double& em1,
                               double inv8f = 1.0 / 40320.0) {
  B = fmax(B, -1.0e6);
  const double n = rint(B * kLog2e);
  const double r = fma(-n, kLn2, B);
  double q = fma(inv8f, r, 1.0 / 5040.0);   // 1/8! r + 1/7!
  q = fma(q, r, 1.0 / 720.0);
  q = fma(q, r, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  q = fma(q, r, 1.0);
  eb = ldexp(fma(r, q, 1.0), static_cast<int>(n));
  em1 = eb - 1.0;
}

// e^B and e^B - 1 for B <= 0: B = n ln2 + r, |r| <= ln2/2, e^r - 1 = r q(r)
// with q the Taylor series of (e^r - 1)/r to r^9/10! (truncation ~3e-13).
// For |B| <= ln2/2 (n = 0) e^B - 1 is the series value r q(r) itself, so it
// keeps its relative accuracy however small B is; otherwise it is e^B - 1
// (|e^B - 1| >= 0.29 there). B below -1400 is clamped (e^-1400 underflows FP64
// to 0 either way).
template <bool THREE_ADDR = false>
__device__ inline void exp_em1(double B, double& eb, double& em1) {
  auto mad = [](double x, double y, double z) { return THREE_ADDR ? fma3(x, y, z) : fma(x, y, z); };
  B = fmax(B, -1400.0);
  const double n = rint(B * kLog2e);
  double r = fma(-n, kLn2Hi, B);
  r = fma(-n, kLn2Lo, r);
  double q = 1.0 / 3628800.0;          // 1/10!
  q = mad(q, r, 1.0 / 362880.0);
  q = mad(q, r, 1.0 / 40320.0);
  q = mad(q, r, 1.0 / 5040.0);
  q = mad(q, r, 1.0 / 720.0);
  q = mad(q, r, 1.0 / 120.0);
  q = mad(q, r, 1.0 / 24.0);
  q = mad(q, r, 1.0 / 6.0);
  q = mad(q, r, 0.5);
  q = fma(q, r, 1.0);
  eb = ldexp(fma(r, q, 1.0), static_cast<int>(n));
  em1 = n == 0.0 ? r * q : eb - 1.0;
}

// Nearest int of an integral double, saturated at the int range (the
// conversion instruction's own behaviour, spelled out so that out-of-range
// values are defined).
__device__ __forceinline__ int sat_int(double n) {
  int r;
  asm("v_cvt_i32_f64 %0, %1" : "=v"(r) : "v"(n));
  return r;
}

// e^X as float for X <= 0: y = X log2(e) in FP64 (rounding |y| 1e-16), split
// into its nearest integer n and |f| <= 1/2, then the hardware base-2
// exponential of f and an exact power-of-two scale. Very negative X gives
// 2^f with n saturated far below the FP32 range: 0.
__device__ inline float exp_neg(double X) {
  const double y = X * kLog2e;
  const double n = rint(y);
  const float p = __builtin_amdgcn_exp2f(static_cast<float>(y - n));
  return ldexpf(p, sat_int(n));
}

// sin(pi x/2) and cos(pi x/2) in FP32 for |x| <= 1/2: Taylor series of sine
// to y^9 and cosine to y^10 in y = pi x/2, |y| <= pi/4 (truncation below 2e-8
// relative).
__device__ inline void sincos_halfpi(float x, float& s, float& c) {
  const float y = 1.57079632679489661923f * x;
  const float z = y * y;
  float ps = 1.f / 362880.f;
  ps = fmaf(ps, z, -1.f / 5040.f);
  ps = fmaf(ps, z, 1.f / 120.f);
  ps = fmaf(ps, z, -1.f / 6.f);
  s = fmaf(y * z, ps, y);
  float pc = -1.f / 3628800.f;
  pc = fmaf(pc, z, 1.f / 40320.f);
  pc = fmaf(pc, z, -1.f / 720.f);
  pc = fmaf(pc, z, 1.f / 24.f);
  pc = fmaf(pc, z, -0.5f);
  c = fmaf(z, pc, 1.f);
}

// sin(2 pi t) and cos(2 pi t) in FP64 for any t: t is reduced to the nearest
// integer and quarter turn, leaving |r| <= pi/4 for the Taylor series
// (sine to r^13, cosine to r^14; truncation below 1e-14).
__device__ inline void sincos_turns(double t, double& s, double& c) {
  constexpr double kTwoPi = 6.283185307179586476925286766559005768;
  const double f = t - rint(t);
  const double qd = rint(4.0 * f);
  const double r = (f - 0.25 * qd) * kTwoPi;
  const double z = r * r;
  double ps = 1.0 / 6227020800.0;      // 1/13!
  ps = fma3(ps, z, -1.0 / 39916800.0);
  ps = fma3(ps, z, 1.0 / 362880.0);
  ps = fma3(ps, z, -1.0 / 5040.0);
  ps = fma3(ps, z, 1.0 / 120.0);
  ps = fma3(ps, z, -1.0 / 6.0);
  const double sr = fma(ps * z, r, r);
  double pc = 1.0 / 87178291200.0;     // 1/14!
  pc = fma3(pc, z, -1.0 / 479001600.0);
  pc = fma3(pc, z, 1.0 / 3628800.0);
  pc = fma3(pc, z, -1.0 / 40320.0);
  pc = fma3(pc, z, 1.0 / 720.0);
  pc = fma3(pc, z, -1.0 / 24.0);
  pc = fma3(pc, z, 0.5);
  const double cr = fma(-pc, z, 1.0);
  const int q = static_cast<int>(qd) & 3;
  s = (q == 0) ? sr : (q == 1) ? cr : (q == 2) ? -sr : -cr;
  c = (q == 0) ? cr : (q == 1) ? -sr : (q == 2) ? -cr : sr;
}

// ------------------------------------------- activations (paper's stored values)
// e^B and e^B - 1 with the series of (e^r - 1)/r to r^12/13! (truncation
// ~1e-17): for values that feed the lobe frame or the lobe parameters, whose
// errors the envelope amplifies by up to lam (1 + a). B is clamped to
// [-1400, 700] (beyond, e^B is 0 or overflows FP64 either way).
__device__ inline void exp_full(double B, double& eb, double& em1) {
  B = fmin(fmax(B, -1400.0), 700.0);
  const double n = rint(B * kLog2e);
  double r = fma(-n, kLn2Hi, B);
  r = fma(-n, kLn2Lo, r);
  double q = 1.0 / 6227020800.0;       // 1/13!
  q = fma3(q, r, 1.0 / 479001600.0);
  q = fma3(q, r, 1.0 / 39916800.0);
  q = fma3(q, r, 1.0 / 3628800.0);
  q = fma3(q, r, 1.0 / 362880.0);
  q = fma3(q, r, 1.0 / 40320.0);
  q = fma3(q, r, 1.0 / 5040.0);
  q = fma3(q, r, 1.0 / 720.0);
  q = fma3(q, r, 1.0 / 120.0);
  q = fma3(q, r, 1.0 / 24.0);
  q = fma3(q, r, 1.0 / 6.0);
  q = fma3(q, r, 0.5);
  q = fma(q, r, 1.0);
  eb = ldexp(fma(r, q, 1.0), static_cast<int>(n));
  em1 = eb - 1.0;
}

// tanh u and sech u (= +sqrt(1 - tanh^2 u)) from one exponential q = e^{-|u|}:
// tanh|u| = (1 - q)(1 + q)/(1 + q^2), sech u = 2 q/(1 + q^2); no overflow.
__device__ inline void tanh_sech(double u, double& t, double& s) {
  double q, qm1;
  exp_full(-fabs(u), q, qm1);
  const double inv = rcp64(fma(q, q, 1.0));
  t = copysign(-qm1 * (1.0 + q) * inv, u);
  s = 2.0 * q * inv;
}

// k = 20 (tanh u + 1) = 40/(1 + e^{-2u}) and dk/du = 20 sech^2 u
// = 80 t/(1 + t)^2 with t = e^{-2|u|} (no overflow, no cancellation).
__device__ inline void k_activation(double u, double& k, double& dk) {
  double t, tm1;
  exp_full(-2.0 * fabs(u), t, tm1);
  const double inv = rcp64(1.0 + t);
  k = 40.0 * (u >= 0.0 ? 1.0 : t) * inv;
  dk = 80.0 * t * inv * inv;
}

// ------------------------------------------------------------- normaliser

struct LobeNorm {
  float n;        // normaliser value
  float dl, da;   // d ln N / d lambda, d ln N / d a
  float dk, dz;   // d ln N / d k, d ln N / d zeta (zero for the NASG normaliser)
};

// Psi(Lam, k) = 2 Lam e^{-Lam} S(r) / (1 - e^{-2 Lam}) of the closed-form
// integral (Section 5.1), r = Lam^2 - k^2, S(r) = sinh(sqrt r)/sqrt r (continued
// to r < 0 as sin(sqrt -r)/sqrt -r), and its partials in Lam and k.
//
// r > 1: with s = sqrt r and delta = Lam - s = k^2 / (Lam + s),
//   Psi = (Lam/s) e^{-delta} (1 - e^{-2s}) / (1 - e^{-2 Lam}),
//   d ln Psi/dLam = -k^2/(Lam s^2) + (delta/s)(1 + 2g) + 2 (g - g_Lam),
//   d ln Psi/dk   = (k/s)(1/s - 1 - 2g),    g = e^{-2s}/(1 - e^{-2s}),
//   g - g_Lam = -e^{-2s} expm1(-2 delta) / ((1 - e^{-2s})(1 - e^{-2 Lam})):
//   every term vanishes with k instead of cancelling (Psi = 1 and both
//   partials are 0 at k = 0), which keeps the partials relatively accurate
//   where 1/(1 + cos(zeta) Psi) amplifies them (zeta near pi).
// |r| <= 1: power series of S and S' (to r^9/19!); r < -1: sin t / t with
//   t = sqrt(-r); then Psi and its partials from F = e^{-Lam} S and
//   F' = e^{-Lam} S' directly (no small-k cancellation there: k is close to
//   Lam or above it).
// The two exponentials are shared by the branches: e^{-delta} or e^{-Lam},
// and e^{-2s} or e^{-2 Lam}.
__device__ inline void psi_partials(double L, double k, double iL, double& psi,
                                    double& dpsi_dL, double& dpsi_dk) {
  const double r = (L - k) * (L + k);
  const bool hyp = r > 1.0;
  const double ar = fmax(fabs(r), 1.0);
  const double is = rsqrt64(ar);                   // 1/s, s = sqrt|r| (where |r| > 1)
  const double s = ar * is;
  const double delta = k * k * rcp64(L + s);
  double e1, e1m1, e2, e2m1;
  exp_em1<true>(hyp ? -delta : -L, e1, e1m1);      // e^{-delta} or e^{-Lam}
  exp_em1<true>(hyp ? -2.0 * s : -2.0 * L, e2, e2m1);   // e^{-2s} or e^{-2 Lam}
  if (hyp) {
    const double Ds = -e2m1;                       // 1 - e^{-2s}
    const double e2L = e2 * e1 * e1;               // e^{-2 Lam} = e^{-2s} e^{-2 delta}
    const double DL = 1.0 - e2L;
    const double iDD = rcp64(Ds * DL);
    const double g = e2 * DL * iDD;
    psi = L * is * e1 * Ds * Ds * iDD;
    const double dlnL = fma(-k * k * iL, is * is, delta * is * fma(2.0, g, 1.0)) -
                        2.0 * e2 * e1m1 * (2.0 + e1m1) * iDD;
    const double dlnk = k * is * (is - 1.0 - 2.0 * g);
    dpsi_dL = psi * dlnL;
    dpsi_dk = psi * dlnk;
  } else {
    double F, dF;
    if (!(fabs(r) > 1.0)) {
      // 1/(2n+1)! for n = 0..9
      constexpr double c[10] = {1.0, 1.0 / 6.0, 1.0 / 120.0, 1.0 / 5040.0, 1.0 / 362880.0,
                                1.0 / 39916800.0, 1.0 / 6227020800.0, 1.0 / 1307674368000.0,
                                1.0 / 355687428096000.0, 1.0 / 121645100408832000.0};
      double sr = c[9], ds = 9.0 * c[9];
#pragma unroll
      for (int n = 8; n >= 1; --n) {
        sr = fma3(sr, r, c[n]);
        ds = fma3(ds, r, n * c[n]);
      }
      sr = fma(sr, r, c[0]);
      F = e1 * sr;
      dF = e1 * ds;
    } else {
      double sn, cs;
      sincos_turns(s * kInvTwoPi, sn, cs);
      F = e1 * sn * is;
      dF = e1 * fma(-s, cs, sn) * 0.5 * is * is * is;
    }
    const double iD = rcp64(-e2m1);                // 1 / (1 - e^{-2 Lam})
    psi = 2.0 * L * F * iD;
    const double dF_dL = fma(2.0 * L, dF, -F);
    dpsi_dL = (2.0 * F + 2.0 * L * dF_dL) * iD - 4.0 * L * F * e2 * iD * iD;
    dpsi_dk = -4.0 * L * k * dF * iD;
  }
}

// Normaliser of one lobe and the log-derivatives the backward pass needs.
// mode 0: 1 / closed-form integral (Section 5.1; the phase multiplies Psi by
//         cos zeta): I = pi (1 - e^{-2 lam}) / (lam sqrt(1+a)) B,
//         B = 1 + cos(zeta) Psi, which FP64 keeps relatively accurate down to
//         B ~ 1e-9 (zeta within ~5e-5 of pi with Psi -> 1);
// mode 1: NASG normaliser lambda sqrt(1+a) / (2 pi (1 - e^{-2 lambda})).
__device__ inline LobeNorm lobe_norm(double lam, double a, double kd, double zd, int mode) {
  double e2l, em1_2l;
  exp_em1<true>(-2.0 * lam, e2l, em1_2l);
  const double dlam = -em1_2l;                    // 1 - e^{-2 lam}, relatively accurate
  const double sq = sqrt64(1.0 + a);
  const double idl = rcp64(dlam);
  const double il = rcp64(lam);
  const double ia = rcp64(1.0 + a);
  // d/dlam ln(lam / (1 - e^{-2 lam})) = 1/lam - 2 e^{-2 lam} / (1 - e^{-2 lam})
  const double dl_base = il - 2.0 * e2l * idl;
  const double da_base = 0.5 * ia;
  LobeNorm out;
  if (mode == 1) {
    out.n = static_cast<float>(lam * sq * idl * (0.5 / kPi));
    out.dl = static_cast<float>(dl_base);
    out.da = static_cast<float>(da_base);
    out.dk = 0.f;
    out.dz = 0.f;
    return out;
  }
  const double L = lam * (1.0 + a);
  double psi, dpsi_dL, dpsi_dk;
  psi_partials(L, kd, il * ia, psi, dpsi_dL, dpsi_dk);
  double sz, cz;
  sincos_turns(zd * kInvTwoPi, sz, cz);
  const double B = fma(cz, psi, 1.0);
  const double iB = rcp64(B);
  const double czB = cz * iB;
  out.n = static_cast<float>(lam * sq * idl * iB * (1.0 / kPi));
  out.dl = static_cast<float>(dl_base - czB * dpsi_dL * (1.0 + a));
  out.da = static_cast<float>(da_base - czB * dpsi_dL * lam);
  out.dk = static_cast<float>(-czB * dpsi_dk);
  out.dz = static_cast<float>(sz * psi * iB);
  return out;
}


// ------------------------------------------------ normaliser, FP32 fast path
// The same normaliser and log-derivatives in FP32 for lam >= 1/2 and
// Lam = lam (1 + a) >= 3/2, the range every lobe of a trained model or a
// log-uniform draw in [1, 1e3] falls in; smaller lam or Lam take the FP64
// code above. In that range nothing below cancels by more than a factor of a
// few, so FP32 keeps N relatively accurate to ~1e-6 and the log-derivatives
// to ~1e-6 of their size:
// - 1 - e^{-2 lam} >= 0.63 and d/dlam ln(lam / (1 - e^{-2 lam})) >= 0.84;
// - B = 1 + cos(zeta) Psi is formed as (1 - Psi) + Psi (1 + cos zeta), with
//   sin zeta, cos zeta and 1 + cos zeta each relatively accurate (the phase
//   is reduced in FP64): for 0 <= Psi <= 1 two terms of one sign, for Psi < 0
//   (|Psi| < 0.22) B >= 0.78, so B keeps its relative accuracy as zeta -> pi
//   and k -> 0 drive it to 0, and the k and zeta log-derivatives keep theirs
//   next to the zeros of cos zeta and sin zeta;
// - where Lam^2 - k^2 > 1, with s, delta, g as in psi_partials and
//   m = 1 - e^{-delta} (relatively accurate),
//     1 - Psi = [m (1 + e^{-delta} e^{-2s}) - delta e^{-delta} (1 - e^{-2s})/s]
//               / (1 - e^{-2 Lam}),
//   whose two terms (~delta and ~delta/s) differ by at least a factor s >= 3/2
//   for small k, and the log-derivatives are those of psi_partials with
//   1 - e^{-2 delta} = m (2 - m): every term vanishes with k;
// - elsewhere (|Lam^2 - k^2| <= 1, or k^2 > Lam^2 + 1) k >= 1.1, Psi <= 0.83,
//   and Psi and its partials come from e^{-Lam} S(r) and e^{-Lam} S'(r) as in
//   psi_partials: S and S' by their series to r^6/13! (both positive there),
//   or, where k^2 > Lam^2 + 1, sin t / t and its derivative in FP64, since
//   they cross zero and the k and zeta gradients scale with them.

__device__ inline float exp_f(float x) { return __builtin_amdgcn_exp2f(x * 1.44269504088896341f); }

// e^x - 1 for x <= 0, relatively accurate: the Taylor series to x^8/8! for
// x > -1/2 (truncation below 1e-8 relative), e^x - 1 below (|e^x - 1| >= 0.39).
__device__ inline float expm1_neg_f(float x) {
  float p = 1.f / 40320.f;
  p = fmaf(p, x, 1.f / 5040.f);
  p = fmaf(p, x, 1.f / 720.f);
  p = fmaf(p, x, 1.f / 120.f);
  p = fmaf(p, x, 1.f / 24.f);
  p = fmaf(p, x, 1.f / 6.f);
  p = fmaf(p, x, 0.5f);
  p = fmaf(p, x, 1.f);
  return x > -0.5f ? p * x : exp_f(x) - 1.f;
}

// sin, cos and 1 + cos of (pi/2) x for x given in FP64: x is split into its
// nearest integer n (the quadrant) and the exact offset |g| <= 1/2, so all
// three stay relatively accurate next to their zeros (1 + cos near x = 2 is
// formed as 1 - cos(pi g/2) from the cosine series itself).
__device__ inline void sincos_phase(double x, float& s, float& c, float& opc) {
  const double n = rint(x);
  const float y = 1.57079632679489661923f * static_cast<float>(x - n);
  const float z = y * y;
  float ps = 1.f / 362880.f;
  ps = fmaf(ps, z, -1.f / 5040.f);
  ps = fmaf(ps, z, 1.f / 120.f);
  ps = fmaf(ps, z, -1.f / 6.f);
  const float sy = fmaf(y * z, ps, y);
  float pc = -1.f / 3628800.f;
  pc = fmaf(pc, z, 1.f / 40320.f);
  pc = fmaf(pc, z, -1.f / 720.f);
  pc = fmaf(pc, z, 1.f / 24.f);
  pc = fmaf(pc, z, -0.5f);
  const float omc = -z * pc;                           // 1 - cos y
  const float cy = 1.f - omc;
  const int q = sat_int(n) & 3;
  s = (q == 0) ? sy : (q == 1) ? cy : (q == 2) ? -sy : -cy;
  c = (q == 0) ? cy : (q == 1) ? -sy : (q == 2) ? -cy : sy;
  opc = (q == 2) ? omc : 1.f + c;
}

// zh = zeta / pi in FP64 (the carrier's own phase offset); lam, a, k as the
// caller holds them (FP64 for the paper's activated values), rounded to FP32
// here except where the sine branch needs them exact.
__device__ inline LobeNorm lobe_norm_f32(double lamd, double ad, double kd, double zh, int mode) {
  const float lam = static_cast<float>(lamd), a = static_cast<float>(ad), k = static_cast<float>(kd);
  const float e2l = exp_f(-2.f * lam);
  const float idl = __builtin_amdgcn_rcpf(1.f - e2l);
  const float il = __builtin_amdgcn_rcpf(lam);
  const float opa = 1.f + a;
  const float ia = __builtin_amdgcn_rcpf(opa);
  const float sq = opa * __builtin_amdgcn_rsqf(opa);
  const float dl_base = il - 2.f * e2l * idl;
  const float da_base = 0.5f * ia;
  LobeNorm out;
  if (mode == 1) {
    out.n = lam * sq * idl * static_cast<float>(0.5 / kPi);
    out.dl = dl_base;
    out.da = da_base;
    out.dk = 0.f;
    out.dz = 0.f;
    return out;
  }
  const float L = lam * opa;
  const float r = (L - k) * (L + k);
  const bool hyp = r > 1.f;
  const float ar = fmaxf(fabsf(r), 1.f);
  const float is = __builtin_amdgcn_rsqf(ar);          // 1/s
  const float s = ar * is;
  const float delta = k * k * __builtin_amdgcn_rcpf(L + s);
  const float e1 = exp_f(hyp ? -delta : -L);           // e^{-delta} or e^{-Lam}
  const float e2 = exp_f(hyp ? -2.f * s : -2.f * L);   // e^{-2s} or e^{-2 Lam}
  float psi, om, dPL, dPk;
  if (hyp) {
    const float Ds = 1.f - e2;
    const float iDs = __builtin_amdgcn_rcpf(Ds);
    const float iDL = __builtin_amdgcn_rcpf(1.f - e2 * e1 * e1);
    const float g = e2 * iDs;
    psi = L * is * e1 * Ds * iDL;
    const float m = -expm1_neg_f(-delta);              // 1 - e^{-delta}
    om = (m * fmaf(e1, e2, 1.f) - delta * e1 * Ds * is) * iDL;
    const float dlnL = fmaf(-k * k * il * ia, is * is, delta * is * fmaf(2.f, g, 1.f)) +
                       2.f * e2 * (m * (2.f - m)) * iDL * iDs;
    const float dlnk = k * is * (is - 1.f - 2.f * g);
    dPL = psi * dlnL;
    dPk = psi * dlnk;
  } else {
    float S, dS;
    if (!(fabsf(r) > 1.f)) {
      // S(r) = sum r^n/(2n+1)! and S'(r), n <= 6
      S = 1.f / 6227020800.f;
      dS = 6.f / 6227020800.f;
      S = fmaf(S, r, 1.f / 39916800.f);
      dS = fmaf(dS, r, 5.f / 39916800.f);
      S = fmaf(S, r, 1.f / 362880.f);
      dS = fmaf(dS, r, 4.f / 362880.f);
      S = fmaf(S, r, 1.f / 5040.f);
      dS = fmaf(dS, r, 3.f / 5040.f);
      S = fmaf(S, r, 1.f / 120.f);
      dS = fmaf(dS, r, 2.f / 120.f);
      S = fmaf(S, r, 1.f / 6.f);
      dS = fmaf(dS, r, 1.f / 6.f);
      S = fmaf(S, r, 1.f);
    } else {
      // sin t / t and its derivative in r, t = sqrt(k^2 - Lam^2), in FP64:
      // S'(r) = (sin t - t cos t)/(2 t^3) and S itself cross zero, and both
      // must stay relatively accurate there (the k and zeta gradients scale
      // with them); FP32 rounding of t alone would move them by ~1e-6 t
      const double Ld = lamd * (1.0 + ad);
      const double t2 = (kd - Ld) * (kd + Ld);
      const double it = rsqrt64(t2);
      const double t = t2 * it;
      double sn, cs;
      sincos_turns(t * kInvTwoPi, sn, cs);
      S = static_cast<float>(sn * it);
      dS = static_cast<float>(fma(-t, cs, sn) * (0.5 * it * it * it));
    }
    const float F = e1 * S;
    const float dF = e1 * dS;
    const float iD = __builtin_amdgcn_rcpf(1.f - e2);
    psi = 2.f * L * F * iD;
    om = 1.f - psi;
    const float dF_dL = fmaf(2.f * L, dF, -F);
    dPL = fmaf(2.f, F, 2.f * L * dF_dL) * iD - 4.f * L * F * e2 * iD * iD;
    dPk = -4.f * L * k * dF * iD;
  }
  float sz, cz, opc;
  sincos_phase(2.0 * zh, sz, cz, opc);                 // sin, cos and 1 + cos of zeta
  const float B = fmaf(psi, opc, om);
  const float iB = __builtin_amdgcn_rcpf(B);
  const float czB = cz * iB;
  out.n = lam * sq * idl * iB * static_cast<float>(1.0 / kPi);
  out.dl = dl_base - czB * dPL * opa;
  out.da = da_base - czB * dPL * lam;
  out.dk = -czB * dPk;
  out.dz = sz * psi * iB;
  return out;
}

// The FP64 normaliser as a called function: it runs only for the rare lobes
// outside the FP32 range, and kept out of line its FP64 temporaries do not
// count against the calling kernel's register budget.
__device__ __noinline__ LobeNorm lobe_norm_outlined(double lam, double a, double kd, double zd,
                                                    int mode) {
  return lobe_norm(lam, a, kd, zd, mode);
}

// The normaliser by the FP32 path where it applies, by the FP64 one elsewhere.
__device__ inline LobeNorm lobe_norm_any(double lam, double a, double kd, double zd, int mode) {
  const float lf = static_cast<float>(lam), af = static_cast<float>(a);
  if (lf >= 0.5f && lf * (1.f + af) >= 1.5f) return lobe_norm_f32(lam, a, kd, zd * kInvPi, mode);
  return lobe_norm_outlined(lam, a, kd, zd, mode);
}

}  // namespace nasg
