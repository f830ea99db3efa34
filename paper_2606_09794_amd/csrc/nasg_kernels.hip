// NASGabor appearance evaluator: forward, backward and fused forward+backward
// kernels for gfx950.
//
// Work mapping: each primitive owns P consecutive lanes of a wavefront. A
// view chunk of P * VPL views is split into P view slots (slot j holds views
// v0 + j + P*t, t < VPL: the direction, upstream gradient, colour and
// direction-gradient accumulators, in registers). Lobes are taken P at a time
// and lane j owns lobe lc + j: it loads that lobe (structure-of-arrays,
// coalesced across primitives) and prepares its constants once (FP64 frame,
// normaliser and its log-derivatives). Then, P times, every lane evaluates its
// own lobe against the view slot it holds and passes the slot on to the next
// lane of the group (ds_bpermute), so each owned lobe meets every view of the
// chunk and each slot ends back in its home lane. A lobe's gradient sums never
// leave its lane and a view's sums travel with its slot: no cross-lane
// reduction per lobe, no atomics, a fixed summation order.
//
// Numerics: the view direction, the frame axes and the dot products d.x, d.z,
// h = 1 - d.z and 1 - (d.z)^2 = h (2 - h) are FP64 (the lobes reach
// lambda (1 + a) ~ 1e6, where FP32 rounding of d.z alone moves G by ~1e-4);
// the carrier phase is reduced in FP64 to its offset from the nearest peak or
// zero, which keeps the carrier and its derivative relatively accurate at its
// peaks and zeros; the envelope exponent ln(p E) is formed in
// FP64 (exp turns its absolute error into a relative error of G) and only
// its final exponential, the carrier's sine/cosine and all gradient factors
// and accumulations are FP32. The normaliser and its log-derivatives are
// FP64, once per lobe.
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
//   dG/dd   = s_x x + s_z z.
#include <hip/hip_runtime.h>

#include "nasg_device.hpp"
#include "nasg_launch.hpp"

namespace nasg {

// ------------------------------------------------------------ ln table
// ln x for x in [1, 2] at compile time: 2 atanh((x - 1)/(x + 1)) summed until
// the terms vanish (|s| <= 1/3).
constexpr double ce_log(double x) {
  const double s = (x - 1.0) / (x + 1.0), z = s * s;
  double term = s, sum = 0.0;
  for (int i = 0; i < 40; ++i) {
    sum += term / (2 * i + 1);
    term *= z;
  }
  return 2.0 * sum;
}

struct LogTable {
  LogEntry e[kLogEntries];
};

// Bucket j covers m in [1/2 + j/256, 1/2 + (j + 1)/256); c is its centre, or
// 1 for the top bucket. ln c is stored as -ln(1/c) of the rounded 1/c, so that
// ln(m (1/c)) - ln(1/c) is ln m whatever the rounding of 1/c.
constexpr LogTable make_log_table() {
  LogTable t{};
  for (int j = 0; j < kLogEntries; ++j) {
    const double c = (j == kLogEntries - 1) ? 1.0 : 0.5 + (j + 0.5) / (2.0 * kLogEntries);
    const double ic = 1.0 / c;
    t.e[j].inv_c = ic;
    t.e[j].ln_c = -ce_log(ic);
  }
  return t;
}

__constant__ const LogTable kLogTable = make_log_table();

// Copies the ln table into this block's LDS (every thread of the block calls it).
__device__ inline void load_log_table(LogEntry* lds) {
  for (int t = threadIdx.x; t < kLogEntries; t += blockDim.x) lds[t] = kLogTable.e[t];
  __syncthreads();
}

// Byte address, for ds_bpermute, of lane j + 1 (cyclically) of this lane's
// group of P.
template <int P>
__device__ inline int group_next_addr() {
  const int lane = static_cast<int>(threadIdx.x & 63);
  return ((lane & ~(P - 1)) | ((lane + 1) & (P - 1))) << 2;
}

// The value held by lane j + 1 of this lane's group (ds_bpermute; every lane
// of the wavefront must be active).
template <int P>
__device__ inline float group_next(float x, int addr) {
  return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
}

template <int P>
__device__ inline double group_next(double x, int addr) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b & 0xffffffffll));
  const int hi = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) |
                              (static_cast<long long>(lo) & 0xffffffffll));
}

// One primitive-lane-group's work: primitive `prim` (may be >= n for tail
// lanes, which compute on a real primitive and write nothing), lane j of P.
template <int P, int VPL, bool BWD, bool BF16, bool ANG>
__device__ __forceinline__ void nasg_body(const NasgArgs& a, int64_t prim, int j,
                                          const LogEntry* ltab) {
  using S = Store<BF16>;
  const int64_t N = a.n;
  const bool valid = prim < N;
  const int64_t i = valid ? prim : N - 1;  // tail lanes compute on a real primitive, write nothing
  const int V = a.v;
  const int K = a.k;
  const int rot_addr = group_next_addr<P>();

  const float c00 = a.c0[3 * i + 0], c01 = a.c0[3 * i + 1], c02 = a.c0[3 * i + 2];
  double base0, base1, base2;
  if (a.dirs != nullptr) {
    base0 = a.dirs[3 * i + 0];
    base1 = a.dirs[3 * i + 1];
    base2 = a.dirs[3 * i + 2];
  } else {
    base0 = a.means[3 * i + 0];
    base1 = a.means[3 * i + 1];
    base2 = a.means[3 * i + 2];
  }

  for (int v0 = 0; v0 < V; v0 += P * VPL) {
    // gradients of later view chunks accumulate onto the first chunk's
    const bool acc_mode = a.accumulate || v0 > 0;

    // ---- per-view state
    double dd[VPL][3];
    float df[VPL][3], rinv[VPL], gr[VPL][3], col[VPL][3], gdir[VPL][3];
    bool has[VPL];
#pragma unroll
    for (int t = 0; t < VPL; ++t) {
      const int v = v0 + j + P * t;
      has[t] = v < V;
      double e0 = base0, e1 = base1, e2 = base2;
      if (a.dirs == nullptr) {
        const int vc = has[t] ? v : 0;
        e0 -= static_cast<double>(a.cams[3 * vc + 0]);
        e1 -= static_cast<double>(a.cams[3 * vc + 1]);
        e2 -= static_cast<double>(a.cams[3 * vc + 2]);
      }
      const double ri = rsqrt64(e0 * e0 + e1 * e1 + e2 * e2);
      dd[t][0] = e0 * ri;
      dd[t][1] = e1 * ri;
      dd[t][2] = e2 * ri;
      df[t][0] = static_cast<float>(dd[t][0]);
      df[t][1] = static_cast<float>(dd[t][1]);
      df[t][2] = static_cast<float>(dd[t][2]);
      rinv[t] = static_cast<float>(ri);
      col[t][0] = c00;
      col[t][1] = c01;
      col[t][2] = c02;
      gdir[t][0] = gdir[t][1] = gdir[t][2] = 0.f;
      if constexpr (BWD) {
        if (has[t]) {
          const int64_t o = (static_cast<int64_t>(v) * N + i) * 3;
          gr[t][0] = a.grad_rgb[o + 0];
          gr[t][1] = a.grad_rgb[o + 1];
          gr[t][2] = a.grad_rgb[o + 2];
        } else {
          gr[t][0] = gr[t][1] = gr[t][2] = 0.f;
        }
      }
    }

    // ---- lobes, P at a time: lane j owns lobe lc + j. The view slots travel
    // round the lane group (lane j takes over the slot of lane j + 1 after
    // every step), so after P steps every owned lobe has met every view of the
    // chunk and every slot is back in its home lane. A lobe's gradient sums
    // stay in the lane that owns it; a view's colour and direction gradient
    // travel with its slot. A lane with no lobe left (K not a multiple of P)
    // carries a zero normaliser and adds nothing.
    for (int lc = 0; lc < K; lc += P) {
      const bool own = lc + j < K;
      const int lo = own ? lc + j : K - 1;
      const int64_t oi = static_cast<int64_t>(lo) * N + i;
      const float4 q = S::load4(a.quat, oi);
      const float4 sh = S::load4(a.shape, oi);
      float w0 = S::load1(a.rgbw, (static_cast<int64_t>(lo) * 3 + 0) * N + i);
      float w1 = S::load1(a.rgbw, (static_cast<int64_t>(lo) * 3 + 1) * N + i);
      float w2 = S::load1(a.rgbw, (static_cast<int64_t>(lo) * 3 + 2) * N + i);
      double xa0, xa1, xa2, za0, za1, za2, lamd, ad, kd;
      // what the gradient write-out needs besides the sums: the frame's own
      // parameters (f*) and, for the paper's raw values, the derivative of
      // each value's activation
      float f0, f1, f2, f3, f4, f5;
      float dlam_du = 1.f, da_du = 1.f, dk_du = 1.f, dw0 = 1.f, dw1 = 1.f, dw2 = 1.f;
      if constexpr (ANG) {
        // Supplementary C: cosines tanh(u) with sines sqrt(1 - c^2) = sech(u),
        // z = (c_t s_p, s_t s_p, c_p),
        // x = (c_t c_p c_s - s_t s_s, s_t c_p c_s + c_t s_s, -s_p c_s);
        // lam = e^u, a = e^u, k = 20 (tanh u + 1), w = tanh u
        double ct, st, cp, sp, cs, ss;
        tanh_sech(q.x, ct, st);
        tanh_sech(q.y, cp, sp);
        tanh_sech(q.z, cs, ss);
        za0 = ct * sp;
        za1 = st * sp;
        za2 = cp;
        xa0 = ct * cp * cs - st * ss;
        xa1 = st * cp * cs + ct * ss;
        xa2 = -sp * cs;
        double em1, dkd;
        exp_full(sh.x, lamd, em1);
        exp_full(sh.y, ad, em1);
        k_activation(sh.z, kd, dkd);
        double t, sc;
        tanh_sech(w0, t, sc);
        w0 = static_cast<float>(t);
        dw0 = static_cast<float>(sc * sc);
        tanh_sech(w1, t, sc);
        w1 = static_cast<float>(t);
        dw1 = static_cast<float>(sc * sc);
        tanh_sech(w2, t, sc);
        w2 = static_cast<float>(t);
        dw2 = static_cast<float>(sc * sc);
        f0 = static_cast<float>(ct);
        f1 = static_cast<float>(st);
        f2 = static_cast<float>(cp);
        f3 = static_cast<float>(sp);
        f4 = static_cast<float>(cs);
        f5 = static_cast<float>(ss);
        dlam_du = static_cast<float>(lamd);
        da_du = static_cast<float>(ad);
        dk_du = static_cast<float>(dkd);
      } else {
        // frame: x = M_x(q)/|q|^2, z = M_z(q)/|q|^2 (homogeneous rotation of q)
        const double qw = q.x, qx = q.y, qy = q.z, qz = q.w;
        const double ww = qw * qw, xx = qx * qx, yy = qy * qy, zz = qz * qz;
        const double is = rcp64(ww + xx + yy + zz);
        xa0 = (ww + xx - yy - zz) * is;
        xa1 = 2.0 * (qx * qy + qw * qz) * is;
        xa2 = 2.0 * (qx * qz - qw * qy) * is;
        za0 = 2.0 * (qx * qz + qw * qy) * is;
        za1 = 2.0 * (qy * qz - qw * qx) * is;
        za2 = (ww - xx - yy + zz) * is;
        lamd = sh.x;
        ad = sh.y;
        kd = sh.z;
        f0 = q.x;
        f1 = q.y;
        f2 = q.z;
        f3 = q.w;
        f4 = static_cast<float>(is);
        f5 = 0.f;
      }
      const double zd = sh.w;
      const double kh = kd * kInvPi;
      const double zh = zd * kInvPi;
      const LobeNorm nm = lobe_norm(lamd, ad, kd, zd, a.norm);
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
      for (int step = 0; step < P; ++step) {
#pragma unroll
        for (int t = 0; t < VPL; ++t) {
          // Branch-free. A view slot beyond V carries a real direction and a zero
          // upstream gradient, so it adds nothing but its (unwritten) colour; at
          // d = -z (kappa = 0) G and every gradient are forced to 0 and kappa is
          // kept away from 0 where it is inverted.
          const double dxd = dd[t][0] * xa0 + dd[t][1] * xa1 + dd[t][2] * xa2;
          const double dzd = dd[t][0] * za0 + dd[t][1] * za1 + dd[t][2] * za2;
          const double hd = 1.0 - dzd;
          const double opd = 1.0 + dzd;             // 2 kappa
          const bool live = opd > 0.0;
          // 2 kappa kept below 2 - 2^-52 (so kappa -> 1 stays in the top
          // ln-table bucket); kappa = lm 2^(le - 1). The table entry is fetched
          // first, its use comes after the carrier and 1/(1 - (d.z)^2).
          const double opc = fmin(opd, 0x1.fffffffffffffp0);
          int le;
          const double lm = frexp(opc, &le);
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
          const double th = fma(dxd, kh, zh);
          const double nh = rint(th);
          float sa, ca;
          sincospi_quarter(0.5f * static_cast<float>(th - nh), sa, ca);
          const bool peak = (static_cast<int>(nh) & 1) == 0;
          const float cpk = peak ? ca : sa;
          const float car = cpk * cpk;
          const float scp = sa * ca;
          // envelope exponent in FP64: X = 2 lam (E kappa - 1) + tau ln kappa
          const bool pole = !(dend > 0.0);
          const double rden = pole ? 0.0 : rcp64(dend);
          const double ud = dxd * dxd * rden;        // tau / a
          const double taud = and_ * ud;
          __builtin_amdgcn_sched_barrier(0);
          // near kappa = 1 (1 + d.z in [1, 2)) the exact kappa is 1 - h/2 and
          // ((1 + d.z) - 2 + h)/2 is the rounding error of the computed one
          const double Ld = log_finish(lm, le - 1, lt, 0.5 * ((opc - 2.0) + hd));
          const double Ad = taud * Ld;               // ln E
          double Ekd, em1d;
          env_exp(Ad + Ld, Ekd, em1d);               // E kappa and E kappa - 1
          const float pE = exp_neg(fma(two_lamd, em1d, Ad));
          const float Npe = live ? Nn * pE : 0.f;
          const float G = Npe * car;
          col[t][0] = fmaf(w0, G, col[t][0]);
          col[t][1] = fmaf(w1, G, col[t][1]);
          col[t][2] = fmaf(w2, G, col[t][2]);
          if constexpr (BWD) {
            const float L = static_cast<float>(Ld);
            const float LR = pole ? -0.25f : static_cast<float>(Ld * rden);  // ln kappa/(1-(d.z)^2)
            const float u = static_cast<float>(ud);
            const float tau = static_cast<float>(taud);
            const float em1 = static_cast<float>(em1d);
            const float g0 = gr[t][0], g1 = gr[t][1], g2 = gr[t][2];
            const float gG = fmaf(g0, w0, fmaf(g1, w1, g2 * w2));
            acc_w0 = fmaf(g0, G, acc_w0);
            acc_w1 = fmaf(g1, G, acc_w1);
            acc_w2 = fmaf(g2, G, acc_w2);
            const float qG = gG * G;
            acc_G += qG;
            acc_l = fmaf(qG, em1, acc_l);
            const float Ek = 1.f + em1;
            const float T2 = fmaf(two_lam, Ek, 1.f);   // 2 lam E kappa + 1
            acc_a = fmaf(qG * T2 * L, u, acc_a);
            const float Sth = (peak ? -scp : scp) * Npe;      // N p E dc/dtheta
            const float gS = gG * Sth;
            acc_k = fmaf(gS, dx, acc_k);
            acc_z += gS;
            const float GTLR = G * T2 * LR;
            const float sx = fmaf(GTLR, two_an * dx, Sth * kf);
            const float inv2k = __builtin_amdgcn_rcpf(opf);   // 1/(2 kappa)
            const float sz = fmaf(GTLR * tau, 2.f * static_cast<float>(dzd),
                                  G * inv2k * fmaf(fmaf(two_lam, tau, two_lam), Ek, tau));
            const float gsx = gG * sx, gsz = gG * sz;
            ax0 = fmaf(gsx, df[t][0], ax0);
            ax1 = fmaf(gsx, df[t][1], ax1);
            ax2 = fmaf(gsx, df[t][2], ax2);
            az0 = fmaf(gsz, df[t][0], az0);
            az1 = fmaf(gsz, df[t][1], az1);
            az2 = fmaf(gsz, df[t][2], az2);
            gdir[t][0] = fmaf(gsx, xf0, fmaf(gsz, zf0, gdir[t][0]));
            gdir[t][1] = fmaf(gsx, xf1, fmaf(gsz, zf1, gdir[t][1]));
            gdir[t][2] = fmaf(gsx, xf2, fmaf(gsz, zf2, gdir[t][2]));
          }
          // pass this view slot on (this lane takes the slot of lane j + 1) as
          // soon as it is done, so the transfer overlaps the next view's work
          if constexpr (P > 1) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              dd[t][c] = group_next<P>(dd[t][c], rot_addr);
              df[t][c] = group_next<P>(df[t][c], rot_addr);
              col[t][c] = group_next<P>(col[t][c], rot_addr);
              if constexpr (BWD) {
                gr[t][c] = group_next<P>(gr[t][c], rot_addr);
                gdir[t][c] = group_next<P>(gdir[t][c], rot_addr);
              }
            }
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }

      // the owning lane writes its lobe's gradients
      if constexpr (BWD) {
        if (valid && own) {
          const int64_t li = static_cast<int64_t>(lc + j) * N + i;
          if (a.g_shape != nullptr) {
            float4 gs = make_float4(fmaf(nm.dl, acc_G, 2.f * acc_l) * dlam_du,
                                    fmaf(nm.da, acc_G, acc_a) * da_du,
                                    fmaf(nm.dk, acc_G, acc_k) * dk_du, fmaf(nm.dz, acc_G, acc_z));
            float4* dst = reinterpret_cast<float4*>(a.g_shape) + li;
            if (acc_mode) {
              const float4 o = *dst;
              gs.x += o.x; gs.y += o.y; gs.z += o.z; gs.w += o.w;
            }
            *dst = gs;
          }
          if (a.g_quat != nullptr) {
            // (ax, az) = (dL/dx, dL/dz)
            float4 gq;
            if constexpr (ANG) {
              // through the raw values u (dc/du = s^2, ds/du = -c s), which keeps
              // the printed 1/s of Supplementary F's Jacobians out:
              //   dx/du_t = s_t (x_1, -x_0, 0),  dz/du_t = s_t (z_1, -z_0, 0),
              //   dx/du_p = s_p c_s z,           dz/du_p = -s_p e_p,
              //   dx/du_s = s_s (s_s e_p - c_s e_t),
              // e_p = (c_t c_p, s_t c_p, -s_p), e_t = (-s_t, c_t, 0)
              const float ct = f0, st = f1, cp = f2, sp = f3, cs = f4, ss = f5;
              const float ep0 = ct * cp, ep1 = st * cp, ep2 = -sp;
              const float xz = ax0 * zf0 + ax1 * zf1 + ax2 * zf2;
              const float xep = ax0 * ep0 + ax1 * ep1 + ax2 * ep2;
              const float zep = az0 * ep0 + az1 * ep1 + az2 * ep2;
              const float xet = ax1 * ct - ax0 * st;
              gq.x = st * (ax0 * xf1 - ax1 * xf0 + az0 * zf1 - az1 * zf0);
              gq.y = sp * (cs * xz - zep);
              gq.z = ss * (ss * xep - cs * xet);
              gq.w = 0.f;
            } else {
              // dL/dq = (J_x^T gx + J_z^T gz)/|q|^2 - 2 q (x.gx + z.gz)/|q|^2
              const float fw = f0, fx = f1, fy = f2, fz = f3, fis = f4;
              const float rad = 2.f * (xf0 * ax0 + xf1 * ax1 + xf2 * ax2 + zf0 * az0 +
                                       zf1 * az1 + zf2 * az2);
              gq.x = 2.f * (fw * ax0 + fz * ax1 - fy * ax2 + fy * az0 - fx * az1 + fw * az2);
              gq.y = 2.f * (fx * ax0 + fy * ax1 + fz * ax2 + fz * az0 - fw * az1 - fx * az2);
              gq.z = 2.f * (-fy * ax0 + fx * ax1 - fw * ax2 + fw * az0 + fz * az1 - fy * az2);
              gq.w = 2.f * (-fz * ax0 + fw * ax1 + fx * ax2 + fx * az0 + fy * az1 + fz * az2);
              gq.x = (gq.x - rad * fw) * fis;
              gq.y = (gq.y - rad * fx) * fis;
              gq.z = (gq.z - rad * fy) * fis;
              gq.w = (gq.w - rad * fz) * fis;
            }
            float4* dst = reinterpret_cast<float4*>(a.g_quat) + li;
            if (acc_mode) {
              const float4 o = *dst;
              gq.x += o.x; gq.y += o.y; gq.z += o.z; gq.w += o.w;
            }
            *dst = gq;
          }
          if (a.g_rgbw != nullptr) {
            float* dst = a.g_rgbw + static_cast<int64_t>(lc + j) * 3 * N + i;
            float r0 = acc_w0 * dw0, r1 = acc_w1 * dw1, r2 = acc_w2 * dw2;
            if (acc_mode) {
              r0 += dst[0];
              r1 += dst[N];
              r2 += dst[2 * N];
            }
            dst[0] = r0;
            dst[N] = r1;
            dst[2 * N] = r2;
          }
        }
      }
    }

    // ---- per-view colours
    if (a.rgb != nullptr && valid) {
#pragma unroll
      for (int t = 0; t < VPL; ++t) {
        if (!has[t]) continue;
        const int64_t o = (static_cast<int64_t>(v0 + j + P * t) * N + i) * 3;
        a.rgb[o + 0] = col[t][0];
        a.rgb[o + 1] = col[t][1];
        a.rgb[o + 2] = col[t][2];
      }
    }

    // ---- diffuse colour and mean / direction gradients
    if constexpr (BWD) {
      float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gm0 = 0.f, gm1 = 0.f, gm2 = 0.f;
#pragma unroll
      for (int t = 0; t < VPL; ++t) {
        gc0 += gr[t][0];
        gc1 += gr[t][1];
        gc2 += gr[t][2];
        // d = e/|e|: dL/de = (I - d d^T) dL/dd / |e|
        const float pr = df[t][0] * gdir[t][0] + df[t][1] * gdir[t][1] + df[t][2] * gdir[t][2];
        gm0 = fmaf(gdir[t][0] - pr * df[t][0], rinv[t], gm0);
        gm1 = fmaf(gdir[t][1] - pr * df[t][1], rinv[t], gm1);
        gm2 = fmaf(gdir[t][2] - pr * df[t][2], rinv[t], gm2);
      }
      gc0 = group_sum<P>(gc0);
      gc1 = group_sum<P>(gc1);
      gc2 = group_sum<P>(gc2);
      gm0 = group_sum<P>(gm0);
      gm1 = group_sum<P>(gm1);
      gm2 = group_sum<P>(gm2);
      if (valid && j == 0) {
        if (a.g_c0 != nullptr) {
          float* dst = a.g_c0 + 3 * i;
          if (acc_mode) {
            gc0 += dst[0];
            gc1 += dst[1];
            gc2 += dst[2];
          }
          dst[0] = gc0;
          dst[1] = gc1;
          dst[2] = gc2;
        }
        if (a.g_geom != nullptr) {
          float* dst = a.g_geom + 3 * i;
          if (acc_mode) {
            gm0 += dst[0];
            gm1 += dst[1];
            gm2 += dst[2];
          }
          dst[0] = gm0;
          dst[1] = gm1;
          dst[2] = gm2;
        }
      }
    }
  }
}

template <int P, int VPL, bool BWD, bool BF16, bool ANG>
// One lane and one view per primitive run three waves per SIMD (the few spills
// land in the once-per-lobe preparation); the other mappings keep two, where the
// full register budget pays more than a third wave.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(P == 1 && VPL == 1 ? 3 : 2)))
void nasg_kernel(const NasgArgs a) {
  __shared__ LogEntry ltab[kLogEntries];
  load_log_table(ltab);
  const int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  nasg_body<P, VPL, BWD, BF16, ANG>(a, gt / P, static_cast<int>(gt & (P - 1)), ltab);
}

// ------------------------------------------------------- persistent batch

template <int P, int VPL, bool ANG>
__device__ __forceinline__ void batch_tile(const NasgArgs& a, int64_t start, int iters,
                                           const LogEntry* ltab) {
  constexpr int kPrimsPerPass = 256 / P;
  for (int m = 0; m < iters; ++m) {
    const int64_t base = start + static_cast<int64_t>(m) * kPrimsPerPass;
    if (base >= a.n) break;  // uniform across the block
    nasg_body<P, VPL, true, false, ANG>(a, base + threadIdx.x / P,
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
// Two waves per SIMD: the three inlined lane mappings would otherwise need
// more registers than that occupancy allows.
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
      case 1: batch_tile<2, 2, false>(sc.args, item.start, sc.tile_iters, ltab); break;
      case 2: batch_tile<8, 2, false>(sc.args, item.start, sc.tile_iters, ltab); break;
      case 3: batch_tile<1, 1, true>(sc.args, item.start, sc.tile_iters, ltab); break;
      case 4: batch_tile<2, 2, true>(sc.args, item.start, sc.tile_iters, ltab); break;
      default: batch_tile<8, 2, true>(sc.args, item.start, sc.tile_iters, ltab); break;
    }
  }
}

hipError_t launch_batched(const BatchHeader* hdr, const BatchScene* scenes, const BatchItem* items,
                          uint32_t* counter, uint64_t token, int grid, hipStream_t s) {
  hipLaunchKernelGGL(batch_reset, dim3(1), dim3(1), 0, s, counter);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(nasg_batched_kernel, dim3(grid), dim3(256), 0, s, hdr, scenes, items, counter,
                     token);
  return hipGetLastError();
}

// ------------------------------------------------------------ instantiation

template <int P, int VPL, bool BWD, bool BF16, bool ANG>
static hipError_t launch_one(const NasgArgs& a, int block, hipStream_t s) {
  const int64_t threads = a.n * P;
  const int64_t grid = (threads + block - 1) / block;
  hipLaunchKernelGGL((nasg_kernel<P, VPL, BWD, BF16, ANG>), dim3(static_cast<unsigned>(grid)),
                     dim3(block), 0, s, a);
  return hipGetLastError();
}

template <int P, int VPL, bool ANG>
static hipError_t launch_pa(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  if (bwd) return bf16 ? launch_one<P, VPL, true, true, ANG>(a, block, s)
                       : launch_one<P, VPL, true, false, ANG>(a, block, s);
  return bf16 ? launch_one<P, VPL, false, true, ANG>(a, block, s)
              : launch_one<P, VPL, false, false, ANG>(a, block, s);
}

template <int P, int VPL>
static hipError_t launch_pv(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  return a.param == kParamAngles ? launch_pa<P, VPL, true>(a, bwd, bf16, block, s)
                                 : launch_pa<P, VPL, false>(a, bwd, bf16, block, s);
}

hipError_t launch_nasg(const NasgArgs& a, int lanes, int vpl, bool bwd, bool bf16, int block,
                       hipStream_t s) {
#define NASG_CASE(P_, V_) \
  if (lanes == P_ && vpl == V_) return launch_pv<P_, V_>(a, bwd, bf16, block, s);
  NASG_FOR_EACH_CONFIG(NASG_CASE)
#undef NASG_CASE
  return hipErrorInvalidValue;
}

}  // namespace nasg
