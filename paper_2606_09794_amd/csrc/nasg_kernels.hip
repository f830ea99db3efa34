// NASGabor appearance evaluator: forward, backward and fused forward+backward
// kernels for gfx950.
//
// Work mapping: each primitive owns P consecutive lanes of a wavefront; lane j
// evaluates views v = v0 + j + P*t (t < VPL) of that primitive, so one
// primitive's views never leave its lane group. Lobes are taken P at a time:
// lane j loads lobe lc + j (structure-of-arrays, coalesced across primitives)
// and prepares its per-lobe constants (FP64 frame, normaliser and its
// log-derivatives) once; the group then walks those P lobes, reading each
// lobe's constants from the lane that prepared it (ds_bpermute), and loops over
// its own views with the per-view state (direction, upstream gradient, colour
// and direction-gradient accumulators) in registers. Per-lobe gradient partial
// sums are summed over the lane group with DPP row operations; the preparing
// lane keeps its lobe's sums and, once the group has walked the P lobes, every
// lane finalises and writes its own lobe - no atomics, fixed summation order.
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

// Value of lane `src` of this lane's group of P (ds_bpermute; P = 1 is a no-op).
template <int P>
__device__ inline float group_bcast(float x, int src) {
  if constexpr (P == 1) {
    return x;
  } else {
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int addr = ((lane & ~(P - 1)) + src) << 2;
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(x)));
  }
}

template <int P>
__device__ inline double group_bcast(double x, int src) {
  if constexpr (P == 1) {
    return x;
  } else {
    const int lane = static_cast<int>(threadIdx.x & 63);
    const int addr = ((lane & ~(P - 1)) + src) << 2;
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, static_cast<int>(b >> 32));
    return __longlong_as_double((static_cast<long long>(hi) << 32) |
                                (static_cast<long long>(lo) & 0xffffffffll));
  }
}

// One primitive-lane-group's work: primitive `prim` (may be >= n for tail
// lanes, which compute on a real primitive and write nothing), lane j of P.
template <int P, int VPL, bool BWD, bool BF16>
__device__ __forceinline__ void nasg_body(const NasgArgs& a, int64_t prim, int j) {
  using S = Store<BF16>;
  const int64_t N = a.n;
  const bool valid = prim < N;
  const int64_t i = valid ? prim : N - 1;  // tail lanes compute on a real primitive, write nothing
  const int V = a.v;
  const int K = a.k;

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

    // ---- lobes, P at a time: lane j prepares lobe lc + j, the group shares it
    for (int lc = 0; lc < K; lc += P) {
      const int lo = min(lc + j, K - 1);
      const int64_t oi = static_cast<int64_t>(lo) * N + i;
      const float4 q = S::load4(a.quat, oi);
      const float4 sh = S::load4(a.shape, oi);
      const float ow0 = S::load1(a.rgbw, (static_cast<int64_t>(lo) * 3 + 0) * N + i);
      const float ow1 = S::load1(a.rgbw, (static_cast<int64_t>(lo) * 3 + 1) * N + i);
      const float ow2 = S::load1(a.rgbw, (static_cast<int64_t>(lo) * 3 + 2) * N + i);
      // frame: x = M_x(q)/|q|^2, z = M_z(q)/|q|^2 (homogeneous rotation of q)
      const double qw = q.x, qx = q.y, qy = q.z, qz = q.w;
      const double ww = qw * qw, xx = qx * qx, yy = qy * qy, zz = qz * qz;
      const double is = rcp64(ww + xx + yy + zz);
      const double oxa0 = (ww + xx - yy - zz) * is;
      const double oxa1 = 2.0 * (qx * qy + qw * qz) * is;
      const double oxa2 = 2.0 * (qx * qz - qw * qy) * is;
      const double oza0 = 2.0 * (qx * qz + qw * qy) * is;
      const double oza1 = 2.0 * (qy * qz - qw * qx) * is;
      const double oza2 = (ww - xx - yy + zz) * is;
      const double okrev = static_cast<double>(sh.z) * kInvTwoPi;
      const double ozrev = static_cast<double>(sh.w) * kInvTwoPi;
      const LobeNorm nm = lobe_norm(sh.x, sh.y, sh.z, sh.w, a.norm);

      // reduced gradient sums of the lobe this lane prepared
      float k_w0 = 0.f, k_w1 = 0.f, k_w2 = 0.f, k_G = 0.f, k_l = 0.f, k_a = 0.f, k_k = 0.f,
            k_z = 0.f, k_x0 = 0.f, k_x1 = 0.f, k_x2 = 0.f, k_z0 = 0.f, k_z1 = 0.f, k_z2 = 0.f;

      const int nsub = min(P, K - lc);
      for (int s = 0; s < nsub; ++s) {
        const double xa0 = group_bcast<P>(oxa0, s), xa1 = group_bcast<P>(oxa1, s),
                     xa2 = group_bcast<P>(oxa2, s);
        const double za0 = group_bcast<P>(oza0, s), za1 = group_bcast<P>(oza1, s),
                     za2 = group_bcast<P>(oza2, s);
        const double krev = group_bcast<P>(okrev, s), zrev = group_bcast<P>(ozrev, s);
        const float lam = group_bcast<P>(sh.x, s), an = group_bcast<P>(sh.y, s);
        const float kf = group_bcast<P>(sh.z, s);
        const float w0 = group_bcast<P>(ow0, s), w1 = group_bcast<P>(ow1, s),
                    w2 = group_bcast<P>(ow2, s);
        const float Nn = group_bcast<P>(nm.n, s);
        const float two_lam = 2.f * lam;
        const double two_lamd = 2.0 * static_cast<double>(lam);
        const float xf0 = static_cast<float>(xa0), xf1 = static_cast<float>(xa1),
                    xf2 = static_cast<float>(xa2);
        const float zf0 = static_cast<float>(za0), zf1 = static_cast<float>(za1),
                    zf2 = static_cast<float>(za2);

        float acc_w0 = 0.f, acc_w1 = 0.f, acc_w2 = 0.f, acc_G = 0.f, acc_l = 0.f, acc_a = 0.f;
        float acc_k = 0.f, acc_z = 0.f;
        float ax0 = 0.f, ax1 = 0.f, ax2 = 0.f, az0 = 0.f, az1 = 0.f, az2 = 0.f;

#pragma unroll
        for (int t = 0; t < VPL; ++t) {
          // Branch-free. A view slot beyond V carries a real direction and a zero
          // upstream gradient, so it adds nothing but its (unwritten) colour; at
          // d = -z (kappa = 0) G and every gradient are forced to 0 and kappa is
          // kept away from 0 where it is inverted.
          const double dxd = dd[t][0] * xa0 + dd[t][1] * xa1 + dd[t][2] * xa2;
          const double dzd = dd[t][0] * za0 + dd[t][1] * za1 + dd[t][2] * za2;
          const double hd = 1.0 - dzd;
          const double kapd = 0.5 * (1.0 + dzd);
          const bool live = kapd > 0.0;
          const double dend = hd * (2.0 - hd);      // 1 - (d.z)^2
          const float dx = static_cast<float>(dxd);
          const float kap = fmaxf(static_cast<float>(kapd), 1e-30f);
          // carrier phase in revolutions, reduced to the nearest integer
          // (theta = 2 pi (f + integer), |f| <= 1/2). The carrier is cos^2(pi f)
          // and dc/dtheta = -sign(f) sin(pi|f|) cos(pi|f|); both are evaluated
          // from the smaller of |f| and 1/2 - |f| so they stay relatively
          // accurate at the carrier's peaks and zeros alike.
          const double tr = fma(dxd, krev, zrev);
          const double fr = tr - rint(tr);
          const double fa = fabs(fr);
          const bool near_peak = fa <= 0.25;
          float sa, ca;
          sincospi_quarter(static_cast<float>(0.25 - fabs(fa - 0.25)), sa, ca);  // min(|f|, 1/2-|f|)
          const float sin_f = near_peak ? sa : ca;   // sin(pi |f|)
          const float cos_f = near_peak ? ca : sa;   // cos(pi |f|)
          const float car = cos_f * cos_f;
          // envelope exponent in FP64: X = 2 lam (E kappa - 1) + tau ln kappa
          const bool pole = !(dend > 0.0);
          const double rden = pole ? 0.0 : rcp64(dend);
          const double Ld = log_kappa(hd, fmax(kapd, 1e-300));
          const double ud = dxd * dxd * rden;        // tau / a
          const double taud = static_cast<double>(an) * ud;
          const double Ad = taud * Ld;               // ln E
          double Ekd, em1d;
          exp_em1(Ad + Ld, Ekd, em1d);               // E kappa and E kappa - 1
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
            const float fsg = fr < 0.0 ? 1.f : -1.f;          // -sign(f)
            const float Sth = fsg * sin_f * cos_f * Npe;      // N p E dc/dtheta
            const float gS = gG * Sth;
            acc_k = fmaf(gS, dx, acc_k);
            acc_z += gS;
            const float sx = fmaf(G * T2 * LR, 2.f * an * dx, Sth * kf);
            const float inv2k = 0.5f * __builtin_amdgcn_rcpf(kap);
            const float sz = G * (fmaf(two_lam * (1.f + tau), Ek, tau) * inv2k +
                                  T2 * LR * tau * 2.f * static_cast<float>(dzd));
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
        }

        if constexpr (BWD) {
          // group sums (computed by every lane: DPP needs all lanes active);
          // the lane that prepared this lobe keeps them
          const bool mine = (j == s);
#define NASG_KEEP(dst, v)                  \
  {                                        \
    const float sum_ = group_sum<P>(v);    \
    dst = mine ? sum_ : dst;               \
  }
          NASG_KEEP(k_w0, acc_w0);
          NASG_KEEP(k_w1, acc_w1);
          NASG_KEEP(k_w2, acc_w2);
          NASG_KEEP(k_G, acc_G);
          NASG_KEEP(k_l, acc_l);
          NASG_KEEP(k_a, acc_a);
          NASG_KEEP(k_k, acc_k);
          NASG_KEEP(k_z, acc_z);
          NASG_KEEP(k_x0, ax0);
          NASG_KEEP(k_x1, ax1);
          NASG_KEEP(k_x2, ax2);
          NASG_KEEP(k_z0, az0);
          NASG_KEEP(k_z1, az1);
          NASG_KEEP(k_z2, az2);
#undef NASG_KEEP
        }
      }

      // every lane finalises the lobe it prepared (all lanes at once)
      if constexpr (BWD) {
        if (valid && lc + j < K) {
          const int64_t li = static_cast<int64_t>(lc + j) * N + i;
          if (a.g_shape != nullptr) {
            float4 gs = make_float4(fmaf(nm.dl, k_G, 2.f * k_l), fmaf(nm.da, k_G, k_a),
                                    fmaf(nm.dk, k_G, k_k), fmaf(nm.dz, k_G, k_z));
            float4* dst = reinterpret_cast<float4*>(a.g_shape) + li;
            if (acc_mode) {
              const float4 o = *dst;
              gs.x += o.x; gs.y += o.y; gs.z += o.z; gs.w += o.w;
            }
            *dst = gs;
          }
          if (a.g_quat != nullptr) {
            // dL/dq = (J_x^T gx + J_z^T gz)/|q|^2 - 2 q (x.gx + z.gz)/|q|^2
            const float fw = q.x, fx = q.y, fy = q.z, fz = q.w;
            const float fis = static_cast<float>(is);
            const float ox0 = static_cast<float>(oxa0), ox1 = static_cast<float>(oxa1),
                        ox2 = static_cast<float>(oxa2);
            const float oz0 = static_cast<float>(oza0), oz1 = static_cast<float>(oza1),
                        oz2 = static_cast<float>(oza2);
            const float rad = 2.f * (ox0 * k_x0 + ox1 * k_x1 + ox2 * k_x2 + oz0 * k_z0 +
                                     oz1 * k_z1 + oz2 * k_z2);
            float4 gq;
            gq.x = 2.f * (fw * k_x0 + fz * k_x1 - fy * k_x2 + fy * k_z0 - fx * k_z1 + fw * k_z2);
            gq.y = 2.f * (fx * k_x0 + fy * k_x1 + fz * k_x2 + fz * k_z0 - fw * k_z1 - fx * k_z2);
            gq.z = 2.f * (-fy * k_x0 + fx * k_x1 - fw * k_x2 + fw * k_z0 + fz * k_z1 - fy * k_z2);
            gq.w = 2.f * (-fz * k_x0 + fw * k_x1 + fx * k_x2 + fx * k_z0 + fy * k_z1 + fz * k_z2);
            gq.x = (gq.x - rad * fw) * fis;
            gq.y = (gq.y - rad * fx) * fis;
            gq.z = (gq.z - rad * fy) * fis;
            gq.w = (gq.w - rad * fz) * fis;
            float4* dst = reinterpret_cast<float4*>(a.g_quat) + li;
            if (acc_mode) {
              const float4 o = *dst;
              gq.x += o.x; gq.y += o.y; gq.z += o.z; gq.w += o.w;
            }
            *dst = gq;
          }
          if (a.g_rgbw != nullptr) {
            float* dst = a.g_rgbw + static_cast<int64_t>(lc + j) * 3 * N + i;
            float r0 = k_w0, r1 = k_w1, r2 = k_w2;
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

template <int P, int VPL, bool BWD, bool BF16>
__global__ __launch_bounds__(256) void nasg_kernel(const NasgArgs a) {
  const int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  nasg_body<P, VPL, BWD, BF16>(a, gt / P, static_cast<int>(gt & (P - 1)));
}

// ------------------------------------------------------- persistent batch

template <int P, int VPL>
__device__ __forceinline__ void batch_tile(const NasgArgs& a, int64_t start, int iters) {
  constexpr int kPrimsPerPass = 256 / P;
  for (int m = 0; m < iters; ++m) {
    const int64_t base = start + static_cast<int64_t>(m) * kPrimsPerPass;
    if (base >= a.n) break;  // uniform across the block
    nasg_body<P, VPL, true, false>(a, base + threadIdx.x / P, static_cast<int>(threadIdx.x & (P - 1)));
  }
}

__global__ void batch_reset(uint32_t* counter) { *counter = 0u; }

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
  if (hdr->token != token) return;
  const int n_items = hdr->n_items;
  for (;;) {
    if (threadIdx.x == 0) s_item = static_cast<int>(atomicAdd(counter, 1u));
    __syncthreads();
    const int it = s_item;
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem item = items[it];
    const BatchScene& sc = scenes[item.scene];
    switch (sc.variant) {
      case 0: batch_tile<1, 1>(sc.args, item.start, sc.tile_iters); break;
      case 1: batch_tile<2, 2>(sc.args, item.start, sc.tile_iters); break;
      default: batch_tile<8, 2>(sc.args, item.start, sc.tile_iters); break;
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

template <int P, int VPL, bool BWD, bool BF16>
static hipError_t launch_one(const NasgArgs& a, int block, hipStream_t s) {
  const int64_t threads = a.n * P;
  const int64_t grid = (threads + block - 1) / block;
  hipLaunchKernelGGL((nasg_kernel<P, VPL, BWD, BF16>), dim3(static_cast<unsigned>(grid)),
                     dim3(block), 0, s, a);
  return hipGetLastError();
}

template <int P, int VPL>
static hipError_t launch_pv(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  if (bwd) return bf16 ? launch_one<P, VPL, true, true>(a, block, s)
                       : launch_one<P, VPL, true, false>(a, block, s);
  return bf16 ? launch_one<P, VPL, false, true>(a, block, s)
              : launch_one<P, VPL, false, false>(a, block, s);
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
