// NASGabor appearance evaluator: forward, backward and fused forward+backward
// kernels for gfx950.
//
// Work mapping: each primitive owns P consecutive lanes of a wavefront. A
// view chunk of P * VPL views is split into P view slots (slot j holds views
// v0 + j + P*t, t < VPL: the direction, upstream gradient, colour and
// direction-gradient accumulators, in registers). Lobes are taken P at a time
// and lane j owns lobe lc + j: it loads that lobe (structure-of-arrays,
// coalesced across primitives) and prepares its constants once (the FP64 frame,
// normaliser and its log-derivatives). Then, P times, every lane evaluates its
// own lobe against the view slot it holds and passes the slot on to the next
// lane of the group (ds_bpermute), so each owned lobe meets every view of the
// chunk and each slot ends back in its home lane. A lobe's gradient sums never
// leave its lane and a view's sums travel with its slot: no cross-lane
// reduction per lobe, no atomics, a fixed summation order.
//
// Numerics: the view direction, the frame axes, d.x, the squared chord
// |d + z|^2 = 4 kappa (relatively accurate next to the antipode, where
// 1 + d.z would cancel), h = 1 - d.z and 1 - (d.z)^2 are FP64 (the lobes reach
// lambda (1 + a) ~ 1e6, where FP32 rounding of d.z alone moves G by ~1e-4);
// the carrier phase is reduced in FP64 to its offset from the nearest peak or
// zero, which keeps the carrier and its derivative relatively accurate at its
// peaks and zeros; the envelope exponent ln(p E) is formed in
// FP64 (exp turns its absolute error into a relative error of G) and only
// its final exponential, the carrier's sine/cosine and all gradient factors
// and accumulations are FP32. The normaliser and its log-derivatives are
// formed once per lobe: in FP32 where lam >= 1/2 and lam (1 + a) >= 3/2
// (with the cancellation-prone pieces in FP64), in FP64 elsewhere.
//
// Value (Section 5.1): G = N p E c, kappa = (d.z + 1)/2,
//   tau = a (d.x)^2 / (1 - (d.z)^2), E = kappa^tau, p = exp(2 lam (E kappa - 1)),
//   c = (1 + cos(k d.x + zeta)) / 2.
// Gradients (Supplementary F): with ln kappa = L and E kappa = 1 + em1,
//   dG/dlam = 2 G em1 + G dlnN/dlam            (dp/dlam = 2 p (E kappa - 1))
//   dG/da   = G (2 lam E kappa + 1) L dtau/da + G dlnN/da
//   dG/dk   = N p E dc/dk + G dlnN/dk,  dG/dzeta = N p E dc/dzeta + G dlnN/dzeta
//   dG/dx   = s_x d,  s_x = G (2 lam E kappa + 1) L 2 a d.x/(1-(d.z)^2) + k N p E dc/dtheta
//   dG/dz   = s_z d,  s_z = G [lam (1+tau) E + tau/(2 kappa)
//                             + (2 lam E kappa + 1) L tau 2 d.z/(1-(d.z)^2)]
//                         = G [(2 lam E kappa + 1) tau Q + lam E],
//                       Q = 1/(2 kappa) + 2 d.z L/(1-(d.z)^2)  (formed in FP64)
//   dG/dd   = s_x x + s_z z.
#include <hip/hip_runtime.h>

#include "nasg_device.hpp"
#include "nasg_launch.hpp"
#include "nasg_skeleton.hpp"

#ifndef NASG_BC_WAVES
#define NASG_BC_WAVES 3
#endif

namespace nasg {

// The paper's raw lobe values activated (Supplementary C): lam = e^u,
// a = e^u, k = 20 (tanh u + 1), w = tanh u, with the derivatives of k and w.
// A called function: once per lobe, and kept out of line its FP64 series do
// not count against the evaluating kernel's registers.
struct Activated {
  double lam, a, k;
  float dk;
  float w[3], dw[3];
};
__device__ __noinline__ Activated activate_raw(float4 sh, float w0, float w1, float w2, bool car) {
  Activated r;
  double em1, dkd = 0.0;
  exp_full(sh.x, r.lam, em1);
  exp_full(sh.y, r.a, em1);
  r.k = 0.0;
  if (car) k_activation(sh.z, r.k, dkd);
  r.dk = static_cast<float>(dkd);
  const float w[3] = {w0, w1, w2};
  for (int c = 0; c < 3; ++c) {
    double t, sc;
    tanh_sech(w[c], t, sc);
    r.w[c] = static_cast<float>(t);
    r.dw[c] = static_cast<float>(sc * sc);
  }
  return r;
}

// One primitive-lane-group's work: primitive `prim` (may be >= n for tail
// lanes, which compute on a real primitive and write nothing), lane j of P.
// NOCAR: the NASG lobe (Supplementary E): no carrier (k = zeta = 0) and the
// NASG normaliser, which is exact for it.
// BC (views broadcast): the P lanes of a primitive own its lobes as usual but
// every lane holds the same VPL views, so each lane evaluates its lobes
// against all of them with no slot transfer, and the per-view colour and
// direction-gradient partials are summed over the lane group at the end (DPP).
// For few views this spreads a primitive over P lanes (P lobes prepared and
// loaded at once) instead of one lane walking all of them.
template <int P, int VPL, bool BWD, bool BF16, bool ANG, bool NOCAR = false, bool BC = false,
          bool ONCE = false, bool PF = !(P == 1 && VPL == 1)>
__device__ __forceinline__ void nasg_body(const NasgArgs& a, int64_t prim, int j,
                                          const LogEntry* ltab) {
  using S = Store<BF16>;
  const int64_t N = a.n;
  const bool valid = prim < N;
  const int64_t i = valid ? prim : N - 1;  // tail lanes compute on a real primitive, write nothing
  const int V = a.v;
  const int K = a.k;
  const int rot_addr = group_next_addr<P>();
  const double k_third = vreg_const(1.0 / 3.0);
  const double k_inv8f = vreg_const(1.0 / 40320.0);

  const float c0v[3] = {a.c0[3 * i + 0], a.c0[3 * i + 1], a.c0[3 * i + 2]};
  const float* bp = a.dirs != nullptr ? a.dirs : a.means;
  const double base[3] = {bp[3 * i + 0], bp[3 * i + 1], bp[3 * i + 2]};

  for (int v0 = 0; v0 < V; v0 += BC ? VPL : P * VPL) {
    // gradients of later view chunks accumulate onto the first chunk's
    const bool acc_mode = a.accumulate || v0 > 0;
    ViewSlots<VPL> sl;
    slots_setup<P, VPL, BWD, BC, ONCE>(a, i, v0, j, base, c0v, sl);

    // ---- lobes, P at a time: lane j owns lobe lc + j. The view slots travel
    // round the lane group (lane j takes over the slot of lane j + 1 after
    // every step), so after P steps every owned lobe has met every view of the
    // chunk and every slot is back in its home lane. A lobe's gradient sums
    // stay in the lane that owns it; a view's colour and direction gradient
    // travel with its slot. A lane with no lobe left (K not a multiple of P)
    // carries a zero normaliser and adds nothing.
    auto load_rec = [&](int lc_, float4& q_, float4& sh_, float& w0_, float& w1_, float& w2_) {
      const int lo_ = lc_ + j < K ? lc_ + j : K - 1;
      const int64_t oi_ = static_cast<int64_t>(lo_) * N + i;
      q_ = S::template load4<ONCE>(a.quat, oi_);
      sh_ = S::template load4<ONCE>(a.shape, oi_);
      w0_ = S::template load1<ONCE>(a.rgbw, (static_cast<int64_t>(lo_) * 3 + 0) * N + i);
      w1_ = S::template load1<ONCE>(a.rgbw, (static_cast<int64_t>(lo_) * 3 + 1) * N + i);
      w2_ = S::template load1<ONCE>(a.rgbw, (static_cast<int64_t>(lo_) * 3 + 2) * N + i);
    };
    // PF: the next lobe group's records are loaded while the current group
    // is evaluated (by default where a lane meets several views per lobe; the
    // single-view mapping has no registers to spare for them at three waves).
    float4 nq, nsh;
    float nw0, nw1, nw2;
    if constexpr (PF) load_rec(0, nq, nsh, nw0, nw1, nw2);
    for (int lc = 0; lc < K; lc += P) {
      const bool own = lc + j < K;
      float4 q, sh;
      float w0, w1, w2;
      if constexpr (PF) {
        q = nq; sh = nsh; w0 = nw0; w1 = nw1; w2 = nw2;
        if (lc + P < K) load_rec(lc + P, nq, nsh, nw0, nw1, nw2);
      } else {
        load_rec(lc, q, sh, w0, w1, w2);
      }
      double xa[3], za[3], lamd, ad, kd;
      // what the gradient write-out needs besides the sums: the frame's own
      // parameters (f) and, for the paper's raw values, the derivative of
      // each value's activation
      float f[6];
      float dlam_du = 1.f, da_du = 1.f, dk_du = 1.f, dw0 = 1.f, dw1 = 1.f, dw2 = 1.f;
      lobe_frame<ANG>(q, xa, za, f);
      if constexpr (ANG) {
        const Activated act = activate_raw(sh, w0, w1, w2, !NOCAR);
        lamd = act.lam;
        ad = act.a;
        kd = act.k;
        w0 = act.w[0];
        w1 = act.w[1];
        w2 = act.w[2];
        dw0 = act.dw[0];
        dw1 = act.dw[1];
        dw2 = act.dw[2];
        dlam_du = static_cast<float>(lamd);
        da_du = static_cast<float>(ad);
        dk_du = act.dk;
      } else {
        lamd = sh.x;
        ad = sh.y;
        kd = NOCAR ? 0.0 : static_cast<double>(sh.z);
      }
      const double xa0 = xa[0], xa1 = xa[1], xa2 = xa[2];
      const double za0 = za[0], za1 = za[1], za2 = za[2];
      const double zd = NOCAR ? 0.0 : static_cast<double>(sh.w);
      const double kh = kd * kInvPi;
      const double zh = zd * kInvPi;
      const LobeNorm nm = lobe_norm_any(lamd, ad, kd, zd, NOCAR ? 1 : a.norm);
      const float Nn = own ? nm.n : 0.f;
      const float kf = static_cast<float>(kd);
      const float two_lam = static_cast<float>(2.0 * lamd);
      const double two_lamd = 2.0 * lamd;
      const double and_ = ad;
      const float two_an = static_cast<float>(2.0 * ad);
      const float xf0 = static_cast<float>(xa0), xf1 = static_cast<float>(xa1),
                  xf2 = static_cast<float>(xa2);
      const float zf0 = static_cast<float>(za0), zf1 = static_cast<float>(za1),
                  zf2 = static_cast<float>(za2);

      // gradient sums of the owned lobe
      float acc_w0 = 0.f, acc_w1 = 0.f, acc_w2 = 0.f, acc_G = 0.f, acc_l = 0.f, acc_a = 0.f;
      float acc_k = 0.f, acc_z = 0.f;
      float ax0 = 0.f, ax1 = 0.f, ax2 = 0.f, az0 = 0.f, az1 = 0.f, az2 = 0.f;

#pragma unroll 2
      for (int step = 0; step < (BC ? 1 : P); ++step) {
#pragma unroll
        for (int t = 0; t < VPL; ++t) {
          // Branch-free. A view slot beyond V carries a real direction and a zero
          // upstream gradient, so it adds nothing but its (unwritten) colour; at
          // d = -z (kappa = 0) G and every gradient are forced to 0 and kappa is
          // kept away from 0 where it is inverted.
          const double dxd = sl.dd[t][0] * xa0 + sl.dd[t][1] * xa1 + sl.dd[t][2] * xa2;
          // q = |d + z|^2 = 2 (1 + d.z) = 4 kappa from the chord: relatively
          // accurate next to the antipode, where 1 + d.z would cancel. Every
          // other quantity derives from q: kappa = q/4 (exact), h = 1 - d.z =
          // 2 - q/2 (exact where q >= 2, Sterbenz), so kappa and h are
          // consistent and the table ln needs no correction for kappa's own
          // rounding. Next to the axis h keeps an absolute error ~2e-16;
          // nothing below is sensitive to h's relative error there (G, s_x
          // and a's gradient depend on tau only through tau ln kappa and ln
          // kappa/(1 - (d.z)^2), s_z through tau Q, all smooth in h).
          const double e0 = sl.dd[t][0] + za0;
          const double e1 = sl.dd[t][1] + za1;
          const double e2 = sl.dd[t][2] + za2;
          const double q = fma(e0, e0, fma(e1, e1, e2 * e2));
          const double hd = fma(q, -0.5, 2.0);
          const double opd = 0.5 * q;                // 2 kappa
          const bool live = q > 0.0;
          // kappa = lm 2^(le - 2). The table entry is fetched first, its use
          // comes after the carrier and 1/(1 - (d.z)^2).
          int le;
          const double lm = frexp(q, &le);
          const LogEntry lt = ltab[log_bucket(lm)];
          __builtin_amdgcn_sched_barrier(0);   // keep the table read ahead of the carrier work
          const double dend = hd * opd;              // 1 - (d.z)^2
          const float dx = static_cast<float>(dxd);
          const float opf = fmaxf(static_cast<float>(opd), 1e-30f);
          // carrier phase theta/pi = (k d.x + zeta)/pi, reduced to the nearest
          // integer n: theta = pi (n + g), |g| <= 1/2. Even n is a carrier peak,
          // c = cos^2(pi g/2); odd n a zero, c = sin^2(pi g/2); dc/dtheta is
          // -sin(pi g/2) cos(pi g/2) at a peak and +sin cos at a zero. The
          // offset g is exact in FP64, so c and dc/dtheta stay relatively
          // accurate at the carrier's peaks and zeros alike.
          float car = 1.f, scp = 0.f;
          bool peak = true;
          if constexpr (!NOCAR) {
            const double th = fma(dxd, kh, zh);
            const double nh = rint(th);
            float sa, ca;
            sincos_halfpi(static_cast<float>(th - nh), sa, ca);
            peak = (static_cast<int>(nh) & 1) == 0;
            const float cpk = peak ? ca : sa;
            car = cpk * cpk;
            scp = sa * ca;
          }
          // envelope exponent in FP64: X = 2 lam (E kappa - 1) + tau ln kappa
          const bool pole = !(dend > 0.0);
          const double rden = pole ? 0.0 : rcp64(dend);
          const double ud = dxd * dxd * rden;        // tau / a
          const double taud = and_ * ud;
          __builtin_amdgcn_sched_barrier(0);
          const double Ld = log_finish(lm, le - 2, lt, 0.0, k_third);
          const double Ad = taud * Ld;               // ln E
          double Ekd, em1d;
          env_exp(Ad + Ld, Ekd, em1d, k_inv8f);      // E kappa and E kappa - 1
          const float pE = exp_neg(fma(two_lamd, em1d, Ad));
          const float Npe = live ? Nn * pE : 0.f;
          const float G = Npe * car;
          sl.col[t][0] = fmaf(w0, G, sl.col[t][0]);
          sl.col[t][1] = fmaf(w1, G, sl.col[t][1]);
          sl.col[t][2] = fmaf(w2, G, sl.col[t][2]);
          if constexpr (BWD) {
            const float LR = pole ? -0.25f : static_cast<float>(Ld * rden);  // ln kappa/(1-(d.z)^2)
            // Q = 1/(2 kappa) + 2 d.z ln kappa/(1 - (d.z)^2) = (h + 2 d.z ln kappa)/(1 - (d.z)^2)
            // in FP64: its two terms (each ~1/2) cancel next to the axis, where
            // Q -> 3h/8 (0 at d = z, where rden is 0)
            const float Q = static_cast<float>(fma(q - 2.0, Ld, hd) * rden);   // 2 d.z = q - 2
            const float tau = static_cast<float>(taud);
            const float em1 = static_cast<float>(em1d);
            const float g0 = sl.gr[t][0], g1 = sl.gr[t][1], g2 = sl.gr[t][2];
            const float gG = fmaf(g0, w0, fmaf(g1, w1, g2 * w2));
            acc_w0 = fmaf(g0, G, acc_w0);
            acc_w1 = fmaf(g1, G, acc_w1);
            acc_w2 = fmaf(g2, G, acc_w2);
            const float qG = gG * G;
            acc_G += qG;
            acc_l = fmaf(qG, em1, acc_l);
            // E kappa itself, not 1 + (E kappa - 1): near d = -z kappa is small and
            // the FP32 difference would carry its absolute error into E kappa
            const float Ek = static_cast<float>(Ekd);
            const float T2 = fmaf(two_lam, Ek, 1.f);   // 2 lam E kappa + 1
            const float Sth = (peak ? -scp : scp) * Npe;      // N p E dc/dtheta
            const float gS = gG * Sth;
            acc_k = fmaf(gS, dx, acc_k);
            acc_z += gS;
            // qT = dL/dG G (2 lam E kappa + 1); uu = qT LR d.x with
            // LR = ln kappa/(1 - (d.z)^2): a's sum takes uu d.x (ln kappa dtau/da
            // = LR (d.x)^2), and dL/dG s_x = uu 2a + dL/dG N p E dc/dtheta k
            const float qT = qG * T2;
            const float uu = qT * LR * dx;
            acc_a = fmaf(uu, dx, acc_a);
            const float gsx = fmaf(uu, two_an, gS * kf);
            const float inv2k = __builtin_amdgcn_rcpf(opf);   // 1/(2 kappa)
            // dL/dG s_z = dL/dG G [(2 lam E kappa + 1) tau Q + lam E],
            // lam E = 2 lam E kappa / (2 kappa)
            const float gsz = fmaf(qT * tau, Q, qG * (two_lam * Ek * inv2k));
            ax0 = fmaf(gsx, sl.df[t][0], ax0);
            ax1 = fmaf(gsx, sl.df[t][1], ax1);
            ax2 = fmaf(gsx, sl.df[t][2], ax2);
            az0 = fmaf(gsz, sl.df[t][0], az0);
            az1 = fmaf(gsz, sl.df[t][1], az1);
            az2 = fmaf(gsz, sl.df[t][2], az2);
            sl.gdir[t][0] = fmaf(gsx, xf0, fmaf(gsz, zf0, sl.gdir[t][0]));
            sl.gdir[t][1] = fmaf(gsx, xf1, fmaf(gsz, zf1, sl.gdir[t][1]));
            sl.gdir[t][2] = fmaf(gsx, xf2, fmaf(gsz, zf2, sl.gdir[t][2]));
          }
          // pass this view slot on (this lane takes the slot of lane j + 1) as
          // soon as it is done, so the transfer overlaps the next view's work
          if constexpr (P > 1 && !BC) {
            slot_pass<P, VPL, BWD>(sl, t, rot_addr);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }

      // the owning lane writes its lobe's gradients, as streaming data in the
      // ONCE flavour (each written once: acc_mode is false there)
      if constexpr (BWD) {
        if (valid && own) {
          const int64_t li = static_cast<int64_t>(lc + j) * N + i;
          if (a.g_shape != nullptr) {
            put4<ONCE>(a.g_shape, li,
                       make_float4(fmaf(nm.dl, acc_G, 2.f * acc_l) * dlam_du,
                                   fmaf(nm.da, acc_G, acc_a) * da_du,
                                   fmaf(nm.dk, acc_G, acc_k) * dk_du, fmaf(nm.dz, acc_G, acc_z)),
                       acc_mode);
          }
          if (a.g_quat != nullptr) {
            const float xf[3] = {xf0, xf1, xf2}, zf[3] = {zf0, zf1, zf2};
            const float gx[3] = {ax0, ax1, ax2}, gz[3] = {az0, az1, az2};
            put4<ONCE>(a.g_quat, li, frame_grad<ANG>(f, xf, zf, gx, gz), acc_mode);
          }
          if (a.g_rgbw != nullptr)
            put_rgbw<ONCE>(a.g_rgbw, lc + j, N, i, acc_w0 * dw0, acc_w1 * dw1,
                                   acc_w2 * dw2, acc_mode);
        }
      }
    }

    slots_finish<P, VPL, BWD, BC, ONCE>(a, i, valid, v0, j, acc_mode, sl);
  }
}

template <int P, int VPL, bool BWD, bool BF16, bool ANG, bool NOCAR, bool BC, bool ONCE>
// One lane and one view per primitive run three waves per SIMD (the few spills
// land in the once-per-lobe preparation), and so do broadcast views; the other
// mappings keep two, where the full register budget pays more than a third wave.
// ONCE (one lane per primitive only): all views fit in one chunk and nothing
// accumulates onto earlier results, so the lobe records are read and every
// output is written exactly once, all as streaming data.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    BC ? NASG_BC_WAVES : (P == 1 && VPL == 1 ? 3 : 2))))
void nasg_kernel(const NasgArgs a) {
  static_assert(!ONCE || P == 1, "the streaming flavour has one lane per primitive");
  __shared__ LogEntry ltab[kLogEntries];
  load_log_table(ltab);
  const int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  nasg_body<P, VPL, BWD, BF16, ANG, NOCAR, BC, ONCE>(a, gt / P, static_cast<int>(gt & (P - 1)),
                                                     ltab);
}

// ------------------------------------------------------- persistent batch

template <int P, int VPL, bool ANG>
__device__ __forceinline__ void batch_tile(const NasgArgs& a, int64_t start, int iters,
                                           const LogEntry* ltab) {
  constexpr int kPrimsPerPass = 256 / P;
  for (int m = 0; m < iters; ++m) {
    const int64_t base = start + static_cast<int64_t>(m) * kPrimsPerPass;
    if (base >= a.n) break;  // uniform across the block
    nasg_body<P, VPL, true, false, ANG, false, false, false, false>(a, base + threadIdx.x / P,
                                        static_cast<int>(threadIdx.x & (P - 1)), ltab);
  }
}

__global__ void batch_reset(uint32_t* counter) { *counter = 0u; }

// Loads a record that every lane of the wave reads at the same address and
// pins each 32-bit word to a scalar register. Without it the compiler sees an
// index that came through LDS as divergent and keeps the scene's pointers and
// sizes in vector registers, with vector address arithmetic on every access.
template <typename T>
__device__ __forceinline__ T load_uniform(const T* p) {
  static_assert(sizeof(T) % 4 == 0, "record size must be a multiple of 4 bytes");
  constexpr int kWords = sizeof(T) / 4;
  uint32_t w[kWords];
  __builtin_memcpy(w, p, sizeof(T));
#pragma unroll
  for (int i = 0; i < kWords; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

// Pulls tiles from the queue until it is empty; every block exits when the
// head passes n_items. A plan whose token does not match is not run.
// Two waves per SIMD: the inlined lane mappings would otherwise need more
// registers than that occupancy allows. RAW: the plan has scenes with the
// paper's raw values, so the five lane mappings are inlined for both
// parametrisations; without them only the five quaternion mappings are, and
// an item of a raw-value scene, which such a plan never holds, is skipped.
template <bool RAW>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void nasg_batched_kernel(const BatchHeader* hdr,
                                                           const BatchScene* scenes,
                                                           const BatchItem* items,
                                                           uint32_t* counter, uint64_t token) {
  __shared__ int s_item;
  __shared__ LogEntry ltab[kLogEntries];
  if (hdr->token != token) return;
  load_log_table(ltab);
  const int n_items = hdr->n_items;
  for (;;) {
    if (threadIdx.x == 0) s_item = static_cast<int>(atomicAdd(counter, 1u));
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_item);
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem item = load_uniform(items + it);
    const BatchScene sc = load_uniform(scenes + item.scene);
    switch (sc.variant) {
      case 0: batch_tile<1, 1, false>(sc.args, item.start, sc.tile_iters, ltab); break;
      case 1: batch_tile<1, 2, false>(sc.args, item.start, sc.tile_iters, ltab); break;
      case 2: batch_tile<1, 4, false>(sc.args, item.start, sc.tile_iters, ltab); break;
      case 3: batch_tile<4, 2, false>(sc.args, item.start, sc.tile_iters, ltab); break;
      case 4: batch_tile<4, 4, false>(sc.args, item.start, sc.tile_iters, ltab); break;
      default:
        if constexpr (RAW) {
          switch (sc.variant) {
            case 5: batch_tile<1, 1, true>(sc.args, item.start, sc.tile_iters, ltab); break;
            case 6: batch_tile<1, 2, true>(sc.args, item.start, sc.tile_iters, ltab); break;
            case 7: batch_tile<1, 4, true>(sc.args, item.start, sc.tile_iters, ltab); break;
            case 8: batch_tile<4, 2, true>(sc.args, item.start, sc.tile_iters, ltab); break;
            default: batch_tile<4, 4, true>(sc.args, item.start, sc.tile_iters, ltab); break;
          }
        }
        break;
    }
  }
}

hipError_t launch_batched(const BatchHeader* hdr, const BatchScene* scenes, const BatchItem* items,
                          uint32_t* counter, uint64_t token, int grid, bool raw, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (raw) {
    hipLaunchKernelGGL(nasg_batched_kernel<true>, dim3(grid), dim3(256), 0, s, hdr, scenes, items,
                       counter, token);
  } else {
    hipLaunchKernelGGL(nasg_batched_kernel<false>, dim3(grid), dim3(256), 0, s, hdr, scenes, items,
                       counter, token);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------ instantiation

template <int P, int VPL, bool BWD, bool BF16, bool ANG, bool NOCAR, bool BC>
static hipError_t launch_one(const NasgArgs& a, int block, hipStream_t s) {
  const int64_t threads = a.n * P;
  const int64_t grid = (threads + block - 1) / block;
  // The streaming flavour (ONCE): one lane per primitive, so that a wave's
  // accesses cover whole cache lines, and a launch that reads every record
  // and writes every output once: all views in one chunk and no accumulation
  // onto earlier results (so acc_mode is always false in it).
  if constexpr (P == 1) {
    if (!a.accumulate && a.v <= VPL) {
      hipLaunchKernelGGL((nasg_kernel<P, VPL, BWD, BF16, ANG, NOCAR, BC, true>),
                         dim3(static_cast<unsigned>(grid)), dim3(block), 0, s, a);
      return hipGetLastError();
    }
  }
  hipLaunchKernelGGL((nasg_kernel<P, VPL, BWD, BF16, ANG, NOCAR, BC, false>),
                     dim3(static_cast<unsigned>(grid)), dim3(block), 0, s, a);
  return hipGetLastError();
}

template <int P, int VPL, bool ANG, bool NOCAR, bool BC>
static hipError_t launch_pa(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  if (bwd) return bf16 ? launch_one<P, VPL, true, true, ANG, NOCAR, BC>(a, block, s)
                       : launch_one<P, VPL, true, false, ANG, NOCAR, BC>(a, block, s);
  return bf16 ? launch_one<P, VPL, false, true, ANG, NOCAR, BC>(a, block, s)
              : launch_one<P, VPL, false, false, ANG, NOCAR, BC>(a, block, s);
}

template <int P, int VPL, bool NOCAR, bool BC = false>
static hipError_t launch_pv(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  return a.param == kParamAngles ? launch_pa<P, VPL, true, NOCAR, BC>(a, bwd, bf16, block, s)
                                 : launch_pa<P, VPL, false, NOCAR, BC>(a, bwd, bf16, block, s);
}

hipError_t launch_nasg(const NasgArgs& a, int lanes, int vpl, bool bcast, bool bwd, bool bf16,
                       int block, hipStream_t s) {
  if (a.family == kFamNasg) {
    // NASG lobes: the compiled family mappings, chosen by view count
    int fl, fv;
    family_mapping(a.v, fl, fv);
    switch (fl) {
      case 1: return launch_pv<1, 1, true>(a, bwd, bf16, block, s);
      case 2: return launch_pv<2, 2, true>(a, bwd, bf16, block, s);
      case 4: return launch_pv<4, 2, true>(a, bwd, bf16, block, s);
      default: return launch_pv<8, 2, true>(a, bwd, bf16, block, s);
    }
  }
  if (a.family != kFamNasgabor) return launch_family(a, bwd, bf16, block, s);
  if (bcast) {
#define NASG_BC_CASE(P_, V_) \
    if (lanes == P_ && vpl == V_) return launch_pv<P_, V_, false, true>(a, bwd, bf16, block, s);
    NASG_FOR_EACH_BCAST_CONFIG(NASG_BC_CASE)
#undef NASG_BC_CASE
    return hipErrorInvalidValue;
  }
#define NASG_CASE(P_, V_) \
  if (lanes == P_ && vpl == V_) return launch_pv<P_, V_, false>(a, bwd, bf16, block, s);
  NASG_FOR_EACH_CONFIG(NASG_CASE)
#undef NASG_CASE
  return hipErrorInvalidValue;
}

}  // namespace nasg
