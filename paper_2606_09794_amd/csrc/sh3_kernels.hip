// Degree-3 real spherical-harmonics appearance (Section 3.2), the comparison
// model: rgb = sum_{j<16} c_j Y_j(d), forward and backward, same lane mapping
// as the NASGabor kernels (P lanes per primitive, VPL views per lane).
//
// Basis (index l*l + l + m), real orthonormal harmonics from the complex ones
// with the Condon-Shortley phase, written as homogeneous polynomials of the
// unit direction. Constants are the closed-form normalisations:
//   Y0 = 1/(2 sqrt(pi))
//   Y1..3 = sqrt(3/(4pi)) (-y, z, -x)
//   Y4 = sqrt(15/(4pi)) xy, Y5 = -sqrt(15/(4pi)) yz,
//   Y6 = sqrt(5/(16pi)) (2z^2 - x^2 - y^2), Y7 = -sqrt(15/(4pi)) xz,
//   Y8 = sqrt(15/(16pi)) (x^2 - y^2)
//   Y9 = -sqrt(35/(32pi)) y (3x^2 - y^2), Y10 = sqrt(105/(4pi)) xyz,
//   Y11 = -sqrt(21/(32pi)) y (4z^2 - x^2 - y^2),
//   Y12 = sqrt(7/(16pi)) z (2z^2 - 3x^2 - 3y^2),
//   Y13 = -sqrt(21/(32pi)) x (4z^2 - x^2 - y^2),
//   Y14 = sqrt(105/(16pi)) z (x^2 - y^2), Y15 = -sqrt(35/(32pi)) x (x^2 - 3y^2)
// The direction gradient of the homogeneous polynomials is projected onto the
// sphere's tangent plane through d = e/|e|, so the choice of extension off the
// sphere does not matter.
//
// Each Y_j is s_j M_j with s_j its signed normalisation and M_j a polynomial
// with small integer coefficients. The kernels fold s_j into the primitive's
// coefficients as they are loaded (c'_j = s_j c_j), so per view they evaluate
// only the M_j: rgb = sum c'_j M_j, the direction gradient is that of
// sum_j beta'_j M_j with beta'_j = g . c'_j (= s_j g . c_j), and the
// coefficient gradient sum_v g M_j is scaled by s_j once, when it is written.
// The coefficients, read once per launch, are streamed; so are the
// coefficient gradients, colours and upstream gradients with one lane per
// primitive, whose accesses then cover whole cache lines.
#include <hip/hip_runtime.h>

#include "nasg_device.hpp"
#include "nasg_launch.hpp"

namespace nasg {

namespace shc {
constexpr float c0 = 0.28209479177387814f;
constexpr float c1 = 0.48860251190291992f;
constexpr float c2a = 1.0925484305920792f;
constexpr float c2b = 0.31539156525252005f;
constexpr float c2c = 0.54627421529603959f;
constexpr float c3a = 0.59004358992664352f;
constexpr float c3b = 2.8906114426405538f;
constexpr float c3c = 0.45704579946446572f;
constexpr float c3d = 0.37317633259011540f;
constexpr float c3e = 1.4453057213202769f;
}  // namespace shc

// signed normalisation s_j of Y_j = s_j M_j (j a compile-time index in the
// unrolled loops, so every use folds to a literal)
__device__ constexpr float sh_scale(int j) {
  using namespace shc;
  constexpr float s[16] = {c0,  -c1,  c1,  -c1,  c2a, -c2a, c2b, -c2a,
                           c2c, -c3a, c3b, -c3c, c3d, -c3c, c3e, -c3a};
  return s[j];
}

// M_j(x, y, z), the basis without its normalisation
__device__ inline void sh_monomials(float x, float y, float z, float M[16]) {
  const float xx = x * x, yy = y * y, zz = z * z;
  const float d = xx - yy;
  const float t = fmaf(4.f, zz, -(xx + yy));
  M[0] = 1.f;
  M[1] = y;
  M[2] = z;
  M[3] = x;
  M[4] = x * y;
  M[5] = y * z;
  M[6] = fmaf(2.f, zz, -(xx + yy));
  M[7] = x * z;
  M[8] = d;
  M[9] = y * fmaf(3.f, xx, -yy);
  M[10] = M[4] * z;
  M[11] = y * t;
  M[12] = z * fmaf(-3.f, xx + yy, 2.f * zz);
  M[13] = x * t;
  M[14] = z * d;
  M[15] = x * fmaf(-3.f, yy, xx);
}

// grad of P = sum_j b[j] M_j (b[0] does not enter). P is a polynomial over
// the monomials of (x, y, z) of degree <= 3 (the expansions above, term by
// term); each partial derivative is evaluated as
//   dP/dx = Lx + x (2 Qxx + 3 Cxxx x + 2 Cxxy y + 2 Cxxz z)
//              + y (Qxy + Cxyy y + Cxyz z) + z (Qxz + Cxzz z)
// and its counterparts, with the derivative factors folded into the
// coefficients.
__device__ inline void sh_grad(float x, float y, float z, const float b[16], float& gx,
                               float& gy, float& gz) {
  // degree 1 and the mixed degree-2 coefficients are b[3], b[1], b[2] and
  // b[4] (xy), b[5] (yz), b[7] (xz); the squares' coefficients times 2
  const float Dx = 2.f * (b[8] - b[6]);     // 2 Qxx
  const float Dy = -2.f * (b[6] + b[8]);    // 2 Qyy
  const float Dz = 4.f * b[6];              // 2 Qzz
  // degree 3, one coefficient per monomial
  const float Cxxy = fmaf(3.f, b[9], -b[11]);
  const float Cyyy = -(b[9] + b[11]);
  const float Cxyz = b[10];
  const float Cyzz = 4.f * b[11];
  const float Czzz = 2.f * b[12];
  const float Cxxz = fmaf(-3.f, b[12], b[14]);
  const float Cyyz = fmaf(-3.f, b[12], -b[14]);
  const float Cxzz = 4.f * b[13];
  const float Cxxx = b[15] - b[13];
  const float Cxyy = fmaf(-3.f, b[15], -b[13]);
  gx = fmaf(x, fmaf(3.f * Cxxx, x, fmaf(2.f * Cxxy, y, fmaf(2.f * Cxxz, z, Dx))),
            fmaf(y, fmaf(Cxyy, y, fmaf(Cxyz, z, b[4])), fmaf(z, fmaf(Cxzz, z, b[7]), b[3])));
  gy = fmaf(y, fmaf(3.f * Cyyy, y, fmaf(2.f * Cxyy, x, fmaf(2.f * Cyyz, z, Dy))),
            fmaf(x, fmaf(Cxxy, x, fmaf(Cxyz, z, b[4])), fmaf(z, fmaf(Cyzz, z, b[5]), b[1])));
  gz = fmaf(z, fmaf(3.f * Czzz, z, fmaf(2.f * Cyzz, y, fmaf(2.f * Cxzz, x, Dz))),
            fmaf(x, fmaf(Cxxz, x, fmaf(Cxyz, y, b[7])), fmaf(y, fmaf(Cyyz, y, b[5]), b[2])));
}

template <int P, int VPL, bool BWD>
__global__ __launch_bounds__(256) void sh3_kernel(const ShArgs a) {
  const int64_t gt = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t prim = gt / P;
  const int j = static_cast<int>(gt & (P - 1));
  const int64_t N = a.n;
  const bool valid = prim < N;
  const int64_t i = valid ? prim : N - 1;
  const int V = a.v;

  float cf[16][3];
#pragma unroll
  for (int b = 0; b < 16; ++b)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      cf[b][c] = sh_scale(b) * load_once(&a.sh[static_cast<int64_t>(b * 3 + c) * N + i]);

  float gcf[16][3];
  if constexpr (BWD) {
#pragma unroll
    for (int b = 0; b < 16; ++b) gcf[b][0] = gcf[b][1] = gcf[b][2] = 0.f;
  }
  float gm0 = 0.f, gm1 = 0.f, gm2 = 0.f;

  const float* base = (a.dirs != nullptr) ? a.dirs : a.means;
  const float b0 = base[3 * i + 0], b1 = base[3 * i + 1], b2 = base[3 * i + 2];

  // upstream gradients of a view chunk, loaded one chunk ahead of their use
  // so that the load's latency hides behind the current chunk's arithmetic
  float gq[VPL][3];
  auto load_grad = [&](int c0_, float (&g)[VPL][3]) {
#pragma unroll
    for (int t = 0; t < VPL; ++t) {
      const int v = c0_ + j + P * t;
      const int64_t o = (static_cast<int64_t>(v < V ? v : 0) * N + i) * 3;
      g[t][0] = load_if<P == 1>(&a.grad_rgb[o + 0]);
      g[t][1] = load_if<P == 1>(&a.grad_rgb[o + 1]);
      g[t][2] = load_if<P == 1>(&a.grad_rgb[o + 2]);
    }
  };
  if constexpr (BWD) load_grad(0, gq);

  for (int v0 = 0; v0 < V; v0 += P * VPL) {
    float gn[VPL][3];
    if constexpr (BWD) {
      if (v0 + P * VPL < V) load_grad(v0 + P * VPL, gn);
    }
#pragma unroll
    for (int t = 0; t < VPL; ++t) {
      const int v = v0 + j + P * t;
      if (v >= V) continue;
      float e0 = b0, e1 = b1, e2 = b2;
      if (a.dirs == nullptr) {
        e0 -= a.cams[3 * v + 0];
        e1 -= a.cams[3 * v + 1];
        e2 -= a.cams[3 * v + 2];
      }
      // |e| is far from the denormal range (a camera never sits on a mean)
      const float ri = __builtin_amdgcn_rsqf(e0 * e0 + e1 * e1 + e2 * e2);
      const float x = e0 * ri, y = e1 * ri, z = e2 * ri;
      float Y[16];
      sh_monomials(x, y, z, Y);
      const int64_t o = (static_cast<int64_t>(v) * N + i) * 3;
      if (a.rgb != nullptr && valid) {
        float r0 = 0.f, r1 = 0.f, r2 = 0.f;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          r0 = fmaf(cf[b][0], Y[b], r0);
          r1 = fmaf(cf[b][1], Y[b], r1);
          r2 = fmaf(cf[b][2], Y[b], r2);
        }
        store_if<P == 1>(r0, &a.rgb[o + 0]);
        store_if<P == 1>(r1, &a.rgb[o + 1]);
        store_if<P == 1>(r2, &a.rgb[o + 2]);
      }
      if constexpr (BWD) {
        const float g0 = gq[t][0], g1 = gq[t][1], g2 = gq[t][2];
        float beta[16];
        beta[0] = 0.f;
#pragma unroll
        for (int b = 0; b < 16; ++b) {
          gcf[b][0] = fmaf(g0, Y[b], gcf[b][0]);
          gcf[b][1] = fmaf(g1, Y[b], gcf[b][1]);
          gcf[b][2] = fmaf(g2, Y[b], gcf[b][2]);
          if (b > 0) beta[b] = fmaf(g0, cf[b][0], fmaf(g1, cf[b][1], g2 * cf[b][2]));
        }
        float gx, gy, gz;
        sh_grad(x, y, z, beta, gx, gy, gz);
        const float pr = x * gx + y * gy + z * gz;
        gm0 = fmaf(gx - pr * x, ri, gm0);
        gm1 = fmaf(gy - pr * y, ri, gm1);
        gm2 = fmaf(gz - pr * z, ri, gm2);
      }
    }
    if constexpr (BWD) {
#pragma unroll
      for (int t = 0; t < VPL; ++t) {
        gq[t][0] = gn[t][0];
        gq[t][1] = gn[t][1];
        gq[t][2] = gn[t][2];
      }
    }
  }

  if constexpr (BWD) {
#pragma unroll
    for (int b = 0; b < 16; ++b)
#pragma unroll
      for (int c = 0; c < 3; ++c) gcf[b][c] = sh_scale(b) * group_sum<P>(gcf[b][c]);
    gm0 = group_sum<P>(gm0);
    gm1 = group_sum<P>(gm1);
    gm2 = group_sum<P>(gm2);
    if (valid) {
      if (a.g_sh != nullptr) {
        // two loops, so that the overwriting one keeps its streaming stores
        if (a.accumulate) {
#pragma unroll
          for (int b = 0; b < 16; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              if (((b * 3 + c) & (P - 1)) != j) continue;
              a.g_sh[static_cast<int64_t>(b * 3 + c) * N + i] += gcf[b][c];
            }
        } else {
#pragma unroll
          for (int b = 0; b < 16; ++b)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              if (((b * 3 + c) & (P - 1)) != j) continue;
              store_if<P == 1>(gcf[b][c], &a.g_sh[static_cast<int64_t>(b * 3 + c) * N + i]);
            }
        }
      }
      if (a.g_geom != nullptr && j == 0) {
        float* dst = a.g_geom + 3 * i;
        if (a.accumulate) {
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

template <int P, int VPL, bool BWD>
static hipError_t launch_sh_one(const ShArgs& a, int block, hipStream_t s) {
  const int64_t threads = a.n * P;
  const int64_t grid = (threads + block - 1) / block;
  hipLaunchKernelGGL((sh3_kernel<P, VPL, BWD>), dim3(static_cast<unsigned>(grid)), dim3(block), 0,
                     s, a);
  return hipGetLastError();
}

hipError_t launch_sh(const ShArgs& a, int lanes, int vpl, bool bwd, int block, hipStream_t s) {
#define SH_CASE(P_, V_)                                                              \
  if (lanes == P_ && vpl == V_)                                                      \
    return bwd ? launch_sh_one<P_, V_, true>(a, block, s) : launch_sh_one<P_, V_, false>(a, block, s);
  NASG_FOR_EACH_CONFIG(SH_CASE)
#undef SH_CASE
  return hipErrorInvalidValue;
}

}  // namespace nasg
