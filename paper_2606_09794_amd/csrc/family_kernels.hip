// Lobes of the other families of the paper's distribution table
// (Supplementary A), on the same per-primitive skeleton as the NASGabor
// kernel (travelling view slots, lobe-owning lanes, no atomics):
//
//   SG  : G = c e^{lam (z.d - 1)},          c = lam / (2 pi (1 - e^{-2 lam})),  shape (lam)
//   SB  : G = c (z.d)^beta on z.d > 0,      c = (beta + 1) / (2 pi)
//         (the hemisphere normalisation of Supplementary D),                  shape (beta)
//   SC  : G = c ((1 - rho^2) / (1 + rho^2 - 2 rho z.d))^2,   c = 1/(4 pi),   shape (rho)
//         (the cited spherical Cauchy; the table's "1 - rho^2 - 2 rho z.d" is
//         not a density)
//   ASG : G = max(z.d, 0) e^{-mu (x.d)^2 - lam (y.d)^2},  y = z x x,
//         no normaliser (the table gives none),                               shape (mu, lam)
//
// Per lobe-view the kernel forms G and its partials: dG/d(shape values) and
// the scalars s_x, s_y, s_z with dG/dx = s_x d, dG/dy = s_y d, dG/dz = s_z d,
// so that dG/dd = s_x x + s_y y + s_z z; through y = z x x, dL/dy adds
// dL/dy x z to dL/dx and x x dL/dy to dL/dz. Geometry (directions, frame,
// dot products, 1 - z.d) and every exponent are FP64 for the same reason as
// in the NASGabor kernel (sharp lobes turn an absolute error of the exponent
// into a relative error of G); the final exponential and all gradient
// factors and sums are FP32.
#include <hip/hip_runtime.h>

#include "nasg_device.hpp"
#include "nasg_launch.hpp"
#include "nasg_skeleton.hpp"

namespace nasg {

template <int P, int VPL, bool BWD, bool BF16, int FAM>
__device__ __forceinline__ void family_body(const NasgArgs& a, int64_t prim, int j,
                                            const LogEntry* ltab) {
  using S = Store<BF16>;
  const int64_t N = a.n;
  const bool valid = prim < N;
  const int64_t i = valid ? prim : N - 1;  // tail lanes compute on a real primitive, write nothing
  const int V = a.v;
  const int K = a.k;
  const int rot_addr = group_next_addr<P>();
  const float c0v[3] = {a.c0[3 * i + 0], a.c0[3 * i + 1], a.c0[3 * i + 2]};
  const float* bp = a.dirs != nullptr ? a.dirs : a.means;
  const double base[3] = {bp[3 * i + 0], bp[3 * i + 1], bp[3 * i + 2]};

  for (int v0 = 0; v0 < V; v0 += P * VPL) {
    const bool acc_mode = a.accumulate || v0 > 0;
    ViewSlots<VPL> sl;
    slots_setup<P, VPL, BWD>(a, i, v0, j, base, c0v, sl);

    for (int lc = 0; lc < K; lc += P) {
      const bool own = lc + j < K;
      const int lo = own ? lc + j : K - 1;
      const int64_t oi = static_cast<int64_t>(lo) * N + i;
      const int64_t wi = static_cast<int64_t>(lo) * 3 * N + i;
      const float4 q = S::template load4<false>(a.quat, oi);
      const float4 sh = S::template load4<false>(a.shape, oi);
      const float w0 = S::template load1<false>(a.rgbw, wi);
      const float w1 = S::template load1<false>(a.rgbw, wi + N);
      const float w2 = S::template load1<false>(a.rgbw, wi + 2 * N);
      double xa[3], za[3], ya[3] = {0.0, 0.0, 0.0};
      float f[6];
      lobe_frame<false>(q, xa, za, f);
      if constexpr (FAM == kFamAsg) {
        ya[0] = za[1] * xa[2] - za[2] * xa[1];
        ya[1] = za[2] * xa[0] - za[0] * xa[2];
        ya[2] = za[0] * xa[1] - za[1] * xa[0];
      }
      // normaliser c and d ln c / d(shape value 0)
      const double p0 = sh.x, p1 = sh.y;
      float cn = 1.f, dlc0 = 0.f;
      if constexpr (FAM == kFamSg) {
        const LobeNorm nm = lobe_norm(p0, 0.0, 0.0, 0.0, 1);   // lam / (2 pi (1 - e^{-2 lam}))
        cn = nm.n;
        dlc0 = nm.dl;
      } else if constexpr (FAM == kFamSb) {
        cn = static_cast<float>((p0 + 1.0) * (0.5 / kPi));
        dlc0 = static_cast<float>(rcp64(p0 + 1.0));
      } else if constexpr (FAM == kFamSc) {
        cn = static_cast<float>(0.25 / kPi);
      }
      const float Nn = own ? cn : 0.f;
      const float p0f = static_cast<float>(p0), p1f = static_cast<float>(p1);
      // SC: 1 - rho and 1 - rho^2, and the constant part of dG/drho
      const double om = 1.0 - p0;
      const double omr2 = om * (1.0 + p0);
      const float sc_a = static_cast<float>(-4.0 * p0 * rcp64(omr2));
      const float xf[3] = {static_cast<float>(xa[0]), static_cast<float>(xa[1]),
                           static_cast<float>(xa[2])};
      const float yf[3] = {static_cast<float>(ya[0]), static_cast<float>(ya[1]),
                           static_cast<float>(ya[2])};
      const float zf[3] = {static_cast<float>(za[0]), static_cast<float>(za[1]),
                           static_cast<float>(za[2])};

      float acc_w0 = 0.f, acc_w1 = 0.f, acc_w2 = 0.f, acc_G = 0.f, acc_p0 = 0.f, acc_p1 = 0.f;
      float ax[3] = {0.f, 0.f, 0.f}, ay[3] = {0.f, 0.f, 0.f}, az[3] = {0.f, 0.f, 0.f};

#pragma unroll 2
      for (int step = 0; step < P; ++step) {
#pragma unroll
        for (int t = 0; t < VPL; ++t) {
          const double* d = sl.dd[t];
          const double dzd = d[0] * za[0] + d[1] * za[1] + d[2] * za[2];
          const double hd = 1.0 - dzd;
          float G = 0.f, sx = 0.f, sy = 0.f, sz = 0.f, g0 = 0.f, g1 = 0.f;
          if constexpr (FAM == kFamSg) {
            // exponent lam (z.d - 1) = -lam h, FP64
            G = Nn * exp_neg(-p0 * hd);
            sz = p0f * G;
            g0 = -static_cast<float>(hd) * G;
          } else if constexpr (FAM == kFamSb) {
            // (z.d)^beta = e^{beta ln(z.d)} on z.d > 0; ln from the table, with
            // z.d kept in [1e-300, 1 - 2^-53] (its own value near 1 is exact)
            const bool live = dzd > 0.0;
            const double tc = fmin(fmax(dzd, 1e-300), 0x1.fffffffffffffp-1);
            int le;
            const double lm = frexp(tc, &le);
            const LogEntry lt = ltab[log_bucket(lm)];
            // near 1, (z.d - 1) + h is 0 or the cap's own offset when z.d rounds
            // to 1 (both differences exact there)
            const double lnt = log_finish(lm, le, lt, dzd > 0.5 ? (tc - 1.0) + hd : 0.0);
            const float e = exp_neg(p0 * lnt);
            G = live ? Nn * e : 0.f;
            // dG/d(z.d) = beta G / z.d (z.d floored in FP32, so an underflowed G
            // never meets an infinite reciprocal)
            sz = live ? p0f * G * __builtin_amdgcn_rcpf(fmaxf(static_cast<float>(tc), 1e-30f)) : 0.f;
            g0 = static_cast<float>(lnt) * G;
          } else if constexpr (FAM == kFamSc) {
            // u = 1 + rho^2 - 2 rho z.d = (1 - rho)^2 + 2 rho h, no cancellation
            const double u = fma(om, om, 2.0 * p0 * hd);
            const double iu = rcp64(u);
            const double qd = omr2 * iu;
            G = Nn * static_cast<float>(qd * qd);
            const float iuf = static_cast<float>(iu);
            sz = 4.f * p0f * G * iuf;
            // dG/drho = G [-4 rho/(1 - rho^2) - 4 (rho - z.d)/u], rho - z.d = h - (1 - rho)
            g0 = G * fmaf(-4.f * static_cast<float>(hd - om), iuf, sc_a);
          } else if constexpr (FAM == kFamAsg) {
            const double dxd = d[0] * xa[0] + d[1] * xa[1] + d[2] * xa[2];
            const double dyd = d[0] * ya[0] + d[1] * ya[1] + d[2] * ya[2];
            const float e = exp_neg(-(p0 * dxd * dxd + p1 * dyd * dyd));
            const bool live = dzd > 0.0;
            const float dx = static_cast<float>(dxd), dy = static_cast<float>(dyd);
            G = live ? Nn * static_cast<float>(dzd) * e : 0.f;
            sz = live ? Nn * e : 0.f;
            sx = -2.f * p0f * dx * G;
            sy = -2.f * p1f * dy * G;
            g0 = -dx * dx * G;
            g1 = -dy * dy * G;
          }
          sl.col[t][0] = fmaf(w0, G, sl.col[t][0]);
          sl.col[t][1] = fmaf(w1, G, sl.col[t][1]);
          sl.col[t][2] = fmaf(w2, G, sl.col[t][2]);
          if constexpr (BWD) {
            const float r0 = sl.gr[t][0], r1 = sl.gr[t][1], r2 = sl.gr[t][2];
            const float gG = fmaf(r0, w0, fmaf(r1, w1, r2 * w2));
            acc_w0 = fmaf(r0, G, acc_w0);
            acc_w1 = fmaf(r1, G, acc_w1);
            acc_w2 = fmaf(r2, G, acc_w2);
            acc_G = fmaf(gG, G, acc_G);
            acc_p0 = fmaf(gG, g0, acc_p0);
            acc_p1 = fmaf(gG, g1, acc_p1);
            const float gsx = gG * sx, gsy = gG * sy, gsz = gG * sz;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const float dc = sl.df[t][c];
              az[c] = fmaf(gsz, dc, az[c]);
              if constexpr (FAM == kFamAsg) {
                ax[c] = fmaf(gsx, dc, ax[c]);
                ay[c] = fmaf(gsy, dc, ay[c]);
                sl.gdir[t][c] = fmaf(gsx, xf[c], fmaf(gsy, yf[c], fmaf(gsz, zf[c], sl.gdir[t][c])));
              } else {
                sl.gdir[t][c] = fmaf(gsz, zf[c], sl.gdir[t][c]);
              }
            }
          }
          if constexpr (P > 1) {
            slot_pass<P, VPL, BWD>(sl, t, rot_addr);
            __builtin_amdgcn_sched_barrier(0);
          }
        }
      }

      if constexpr (BWD) {
        if (valid && own) {
          const int64_t li = static_cast<int64_t>(lc + j) * N + i;
          if (a.g_shape != nullptr)
            put4<false>(a.g_shape, li, make_float4(fmaf(dlc0, acc_G, acc_p0), acc_p1, 0.f, 0.f),
                        acc_mode);
          if (a.g_quat != nullptr) {
            float gx[3] = {ax[0], ax[1], ax[2]}, gz[3] = {az[0], az[1], az[2]};
            if constexpr (FAM == kFamAsg) {
              // y = z x x: dL/dx += dL/dy x z, dL/dz += x x dL/dy
              gx[0] += ay[1] * zf[2] - ay[2] * zf[1];
              gx[1] += ay[2] * zf[0] - ay[0] * zf[2];
              gx[2] += ay[0] * zf[1] - ay[1] * zf[0];
              gz[0] += xf[1] * ay[2] - xf[2] * ay[1];
              gz[1] += xf[2] * ay[0] - xf[0] * ay[2];
              gz[2] += xf[0] * ay[1] - xf[1] * ay[0];
            }
            put4<false>(a.g_quat, li, frame_grad<false>(f, xf, zf, gx, gz), acc_mode);
          }
          if (a.g_rgbw != nullptr)
            put_rgbw<false>(a.g_rgbw, lc + j, N, i, acc_w0, acc_w1, acc_w2, acc_mode);
        }
      }
    }
    slots_finish<P, VPL, BWD>(a, i, valid, v0, j, acc_mode, sl);
  }
}

template <int P, int VPL, bool BWD, bool BF16, int FAM>
__global__ __launch_bounds__(256) void family_kernel(const NasgArgs a) {
  __shared__ LogEntry ltab[kLogEntries];
  load_log_table(ltab);
  const int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  family_body<P, VPL, BWD, BF16, FAM>(a, gt / P, static_cast<int>(gt & (P - 1)), ltab);
}

template <int P, int VPL, int FAM>
static hipError_t launch_f(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  const int64_t threads = a.n * P;
  const dim3 grid(static_cast<unsigned>((threads + block - 1) / block));
  if (bwd) {
    if (bf16) hipLaunchKernelGGL((family_kernel<P, VPL, true, true, FAM>), grid, dim3(block), 0, s, a);
    else hipLaunchKernelGGL((family_kernel<P, VPL, true, false, FAM>), grid, dim3(block), 0, s, a);
  } else {
    if (bf16) hipLaunchKernelGGL((family_kernel<P, VPL, false, true, FAM>), grid, dim3(block), 0, s, a);
    else hipLaunchKernelGGL((family_kernel<P, VPL, false, false, FAM>), grid, dim3(block), 0, s, a);
  }
  return hipGetLastError();
}

template <int FAM>
static hipError_t launch_fam(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  int lanes, vpl;
  family_mapping(a.v, lanes, vpl);
  switch (lanes) {
    case 1: return launch_f<1, 1, FAM>(a, bwd, bf16, block, s);
    case 2: return launch_f<2, 2, FAM>(a, bwd, bf16, block, s);
    case 4: return launch_f<4, 2, FAM>(a, bwd, bf16, block, s);
    default: return launch_f<8, 2, FAM>(a, bwd, bf16, block, s);
  }
}

hipError_t launch_family(const NasgArgs& a, bool bwd, bool bf16, int block, hipStream_t s) {
  switch (a.family) {
    case kFamSg: return launch_fam<kFamSg>(a, bwd, bf16, block, s);
    case kFamSb: return launch_fam<kFamSb>(a, bwd, bf16, block, s);
    case kFamSc: return launch_fam<kFamSc>(a, bwd, bf16, block, s);
    case kFamAsg: return launch_fam<kFamAsg>(a, bwd, bf16, block, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace nasg
