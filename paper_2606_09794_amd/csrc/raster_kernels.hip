// Compositing of the primitives' colours into an image for one camera
// (Section 3.1: C = sum_i T_i alpha_i c_i, alpha_i = sigma_i rho_i,
// T_i = prod_{j<i} (1 - alpha_j)), with the gradients of a loss on the image
// with respect to the per-primitive colours and opacities, which is what the
// appearance backward consumes.
//
// The primitives are 3D Gaussians (mean, per-axis scale, quaternion
// rotation); rho on a pixel's ray is the Gaussian projected onto the image
// plane (the local affine approximation of the perspective map at the mean),
// evaluated at the pixel centre. A primitive reaches a pixel only inside its
// 3-sigma ellipse and only in front of the near plane Z = 0.2; alpha is
// clamped at 0.99; the background is black.
//
// Pipeline (all on the caller's stream, nothing allocated, no host sync):
//   project : per primitive, FP64 pixel mean, inverse 2D covariance, depth and
//             the 16 x 16-pixel tiles its ellipse's bounding box touches;
//   bin     : each primitive appends itself to the lists of those tiles
//             (an atomic cursor per tile, fixed capacity per tile; entries
//             beyond it are dropped and flagged);
//   sort    : per tile, the list is sorted by (depth, primitive index) in
//             LDS (bitonic), which fixes the compositing order;
//   render  : one 256-thread block per tile (one pixel per thread), front to
//             back over the list in chunks staged through LDS. The support
//             test and the quadratic form are FP64 (so both sides of a
//             parity check take the same support decisions), rho = exp(-q/2)
//             is FP32, and the transmittance (with an explicit power-of-two
//             exponent) and the colour sum are FP64: with no early
//             termination a pixel may composite thousands of layers;
//   backward: back to front over the same list, with dC/dc_i = alpha_i T_i
//             and dC/dalpha_i = T_i (c_i - R_{i+1}), R the colour seen from
//             the next layer on in units of its transmittance, built by a
//             convex-combination recursion (no cancellation at any depth),
//             and T_i recovered from the forward's final transmittance. A
//             wavefront (4 x 16 pixels) sums its pixels' terms for a
//             primitive in registers and adds them to FP64 per-primitive
//             accumulators with one atomic per value; a last kernel rounds
//             the accumulators to the float32 outputs.
#include <hip/hip_runtime.h>

#include "../../include/nasg.h"
#include "raster.hpp"

namespace nasg {

constexpr double kNear = 0.2;
constexpr float kClamp = 0.99f;
constexpr double kSupport = 9.0;
constexpr int kChunk = 256;

__global__ void raster_zero(int32_t* cursor, int64_t n_tiles, int32_t* overflow) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t < n_tiles) cursor[t] = 0;
  if (t == 0) *overflow = 0;
}

__global__ void raster_zero_acc(double* acc, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    acc[4 * i + 0] = 0.0;
    acc[4 * i + 1] = 0.0;
    acc[4 * i + 2] = 0.0;
    acc[4 * i + 3] = 0.0;
  }
}

__global__ void raster_finish_grads(const double* acc, float* gc, float* go, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) {
    if (gc != nullptr) {
      gc[3 * i + 0] = static_cast<float>(acc[4 * i + 0]);
      gc[3 * i + 1] = static_cast<float>(acc[4 * i + 1]);
      gc[3 * i + 2] = static_cast<float>(acc[4 * i + 2]);
    }
    if (go != nullptr) go[i] = static_cast<float>(acc[4 * i + 3]);
  }
}

__global__ void raster_project(RasterArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  ProjRec rec{};
  rec.tx0 = 1;  // empty tile range unless the ellipse lands on the image
  rec.tx1 = 0;
  rec.ty0 = 1;
  rec.ty1 = 0;
  const double mx = a.means[3 * i], my = a.means[3 * i + 1], mz = a.means[3 * i + 2];
  const double* R = a.cam_rot;
  const double X = R[0] * mx + R[1] * my + R[2] * mz + a.cam_t[0];
  const double Y = R[3] * mx + R[4] * my + R[5] * mz + a.cam_t[1];
  const double Z = R[6] * mx + R[7] * my + R[8] * mz + a.cam_t[2];
  rec.z = Z;
  if (Z > kNear) {
    const double iz = 1.0 / Z;
    rec.u = a.fx * X * iz + a.cx;
    rec.v = a.fy * Y * iz + a.cy;
    // world rotation of the normalised quaternion
    double qw = a.rots[4 * i], qx = a.rots[4 * i + 1], qy = a.rots[4 * i + 2], qz = a.rots[4 * i + 3];
    const double qn = 1.0 / sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw *= qn;
    qx *= qn;
    qy *= qn;
    qz *= qn;
    const double Rw[9] = {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy),
                          2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx),
                          2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)};
    const double s[3] = {a.scales[3 * i], a.scales[3 * i + 1], a.scales[3 * i + 2]};
    // M = J R_cw R_w S (2 x 3), projected covariance Sigma_2 = M M^T
    const double J0[3] = {a.fx * iz, 0.0, -a.fx * X * iz * iz};
    const double J1[3] = {0.0, a.fy * iz, -a.fy * Y * iz * iz};
    double A0[3], A1[3];
    for (int c = 0; c < 3; ++c) {
      A0[c] = J0[0] * R[c] + J0[1] * R[3 + c] + J0[2] * R[6 + c];
      A1[c] = J1[0] * R[c] + J1[1] * R[3 + c] + J1[2] * R[6 + c];
    }
    double m0[3], m1[3];
    for (int c = 0; c < 3; ++c) {
      m0[c] = (A0[0] * Rw[c] + A0[1] * Rw[3 + c] + A0[2] * Rw[6 + c]) * s[c];
      m1[c] = (A1[0] * Rw[c] + A1[1] * Rw[3 + c] + A1[2] * Rw[6 + c]) * s[c];
    }
    const double sxx = m0[0] * m0[0] + m0[1] * m0[1] + m0[2] * m0[2];
    const double sxy = m0[0] * m1[0] + m0[1] * m1[1] + m0[2] * m1[2];
    const double syy = m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2];
    const double det = sxx * syy - sxy * sxy;
    if (det > 0.0) {
      const double id = 1.0 / det;
      rec.a = syy * id;
      rec.b = -sxy * id;
      rec.c = sxx * id;
      // q <= 9 implies |dx| <= 3 sqrt(sxx) and |dy| <= 3 sqrt(syy); one pixel
      // of margin absorbs rounding; pixel px has its centre at px + 1/2
      const double ex = 3.0 * sqrt(sxx) + 1.0, ey = 3.0 * sqrt(syy) + 1.0;
      const double px0 = fmax(rec.u - ex - 0.5, 0.0), px1 = fmin(rec.u + ex - 0.5, a.width - 1.0);
      const double py0 = fmax(rec.v - ey - 0.5, 0.0), py1 = fmin(rec.v + ey - 0.5, a.height - 1.0);
      if (px0 <= px1 && py0 <= py1) {
        rec.tx0 = static_cast<int32_t>(px0) / kTile;
        rec.tx1 = static_cast<int32_t>(px1) / kTile;
        rec.ty0 = static_cast<int32_t>(py0) / kTile;
        rec.ty1 = static_cast<int32_t>(py1) / kTile;
      }
    }
  }
  a.proj[i] = rec;
}

__global__ void raster_bin(RasterArgs a) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const ProjRec r = a.proj[i];
  for (int ty = r.ty0; ty <= r.ty1; ++ty) {
    for (int tx = r.tx0; tx <= r.tx1; ++tx) {
      const int64_t tile = static_cast<int64_t>(ty) * a.tiles_x + tx;
      const int32_t pos = atomicAdd(a.cursor + tile, 1);
      if (pos < a.cap) {
        a.lists[tile * a.cap + pos] = static_cast<int32_t>(i);
      } else {
        atomicMax(a.overflow, 1);
      }
    }
  }
}

// (depth, index) order; padding entries (index < 0) sort last
__device__ inline bool entry_less(double za, int32_t ia, double zb, int32_t ib) {
  if (ia < 0) return false;
  if (ib < 0) return true;
  return za < zb || (za == zb && ia < ib);
}

__global__ __launch_bounds__(256) void raster_sort(RasterArgs a) {
  extern __shared__ unsigned char smem[];
  const int64_t tile = blockIdx.x;
  const int cnt = min(a.cursor[tile], a.cap);
  int m = 1;
  while (m < cnt) m <<= 1;  // m <= cap_pow2, the LDS arrays' length
  double* kz = reinterpret_cast<double*>(smem);
  int32_t* ki = reinterpret_cast<int32_t*>(kz + a.cap_pow2);
  int32_t* list = a.lists + tile * a.cap;
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    if (t < cnt) {
      const int32_t idx = list[t];
      ki[t] = idx;
      kz[t] = a.proj[idx].z;
    } else {
      ki[t] = -1;
      kz[t] = 0.0;
    }
  }
  __syncthreads();
  for (int k = 2; k <= m; k <<= 1) {
    for (int jj = k >> 1; jj > 0; jj >>= 1) {
      for (int t = threadIdx.x; t < m; t += blockDim.x) {
        const int p = t ^ jj;
        if (p > t) {
          const bool up = (t & k) == 0;
          const bool sw = up ? entry_less(kz[p], ki[p], kz[t], ki[t])
                             : entry_less(kz[t], ki[t], kz[p], ki[p]);
          if (sw) {
            const double z = kz[t];
            kz[t] = kz[p];
            kz[p] = z;
            const int32_t x = ki[t];
            ki[t] = ki[p];
            ki[p] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < cnt; t += blockDim.x) list[t] = ki[t];
}

struct StageEntry {
  double u, v, a, b, c;
  float sigma, c0, c1, c2;
  int32_t idx;
  int32_t pad;
};

__device__ inline float wave_sum(float x) {
  for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Transmittance as t * 2^E (E a multiple of kRenorm, t kept away from the
// bottom of the double range), so a pixel behind thousands of layers keeps
// its exact value for the backward's division-based recovery.
constexpr int kRenorm = 600;

__device__ inline void stage_entry(const RasterArgs& a, const int32_t* list, int e,
                                   StageEntry* slot) {
  const int32_t idx = list[e];
  const ProjRec r = a.proj[idx];
  StageEntry s;
  s.u = r.u;
  s.v = r.v;
  s.a = r.a;
  s.b = r.b;
  s.c = r.c;
  s.sigma = a.opac[idx];
  s.c0 = a.colors[3 * idx];
  s.c1 = a.colors[3 * idx + 1];
  s.c2 = a.colors[3 * idx + 2];
  s.idx = idx;
  s.pad = 0;
  *slot = s;
}

__device__ inline double quad_form(const StageEntry& s, double cxp, double cyp) {
  const double dx = cxp - s.u, dy = cyp - s.v;
  return s.a * dx * dx + 2.0 * s.b * dx * dy + s.c * dy * dy;
}

__global__ __launch_bounds__(256) void raster_render_fwd(RasterArgs a) {
  __shared__ StageEntry stage[kChunk];
  const int64_t tile = blockIdx.x;
  const int tx = static_cast<int>(tile % a.tiles_x), ty = static_cast<int>(tile / a.tiles_x);
  const int px = tx * kTile + static_cast<int>(threadIdx.x % kTile);
  const int py = ty * kTile + static_cast<int>(threadIdx.x / kTile);
  const bool inside = px < a.width && py < a.height;
  const double cxp = px + 0.5, cyp = py + 0.5;
  const int cnt = min(a.cursor[tile], a.cap);
  const int32_t* list = a.lists + tile * a.cap;

  double C0 = 0.0, C1 = 0.0, C2 = 0.0;
  double t = 1.0, pw = 1.0;  // T = t * pw, pw = 2^E
  int E = 0;
  for (int base = 0; base < cnt; base += kChunk) {
    __syncthreads();
    const int e = base + static_cast<int>(threadIdx.x);
    if (e < cnt) stage_entry(a, list, e, &stage[threadIdx.x]);
    __syncthreads();
    const int lim = min(kChunk, cnt - base);
    if (!inside) continue;
    for (int k = 0; k < lim; ++k) {
      const StageEntry& s = stage[k];
      const double q = quad_form(s, cxp, cyp);
      if (q <= kSupport) {
        const float rho = __expf(static_cast<float>(-0.5 * q));
        const float al = fminf(s.sigma * rho, kClamp);
        const double w = static_cast<double>(al) * t * pw;
        C0 = fma(w, static_cast<double>(s.c0), C0);
        C1 = fma(w, static_cast<double>(s.c1), C1);
        C2 = fma(w, static_cast<double>(s.c2), C2);
        t *= 1.0 - static_cast<double>(al);
        if (t < 0x1p-600) {
          t *= 0x1p600;
          E -= kRenorm;
          pw = ldexp(1.0, E);
        }
      }
    }
  }
  if (inside) {
    const int64_t pix = static_cast<int64_t>(py) * a.width + px;
    a.image_out[3 * pix] = static_cast<float>(C0);
    a.image_out[3 * pix + 1] = static_cast<float>(C1);
    a.image_out[3 * pix + 2] = static_cast<float>(C2);
    a.pix_state[2 * pix] = t;
    a.pix_state[2 * pix + 1] = static_cast<double>(E);
  }
}

// Back to front over the same sorted list. With R_k the colour seen from
// layer k onwards in units of T_k (R_k = alpha_k c_k + (1 - alpha_k) R_{k+1},
// R = 0 behind the last layer), the colour behind i is S_i = T_i (1 -
// alpha_i) R_{i+1}, so dC/dalpha_i = T_i (c_i - R_{i+1}): no difference of
// large sums, whatever the depth. T_i is recovered from the forward's final
// transmittance, T_i = T_{i+1} / (1 - alpha_i).
__global__ __launch_bounds__(256) void raster_render_bwd(RasterArgs a) {
  __shared__ StageEntry stage[kChunk];
  const int64_t tile = blockIdx.x;
  const int tx = static_cast<int>(tile % a.tiles_x), ty = static_cast<int>(tile / a.tiles_x);
  const int px = tx * kTile + static_cast<int>(threadIdx.x % kTile);
  const int py = ty * kTile + static_cast<int>(threadIdx.x / kTile);
  const bool inside = px < a.width && py < a.height;
  const double cxp = px + 0.5, cyp = py + 0.5;
  const int cnt = min(a.cursor[tile], a.cap);
  const int32_t* list = a.lists + tile * a.cap;

  double t = 1.0, pw = 1.0;
  int E = 0;
  double R0 = 0.0, R1 = 0.0, R2 = 0.0;
  float g0 = 0.f, g1 = 0.f, g2 = 0.f;
  if (inside) {
    const int64_t pix = static_cast<int64_t>(py) * a.width + px;
    t = a.pix_state[2 * pix];
    E = static_cast<int>(a.pix_state[2 * pix + 1]);
    pw = ldexp(1.0, E);
    g0 = a.grad_image[3 * pix];
    g1 = a.grad_image[3 * pix + 1];
    g2 = a.grad_image[3 * pix + 2];
  }
  for (int end = cnt; end > 0; end -= kChunk) {
    const int base = max(0, end - kChunk);
    __syncthreads();
    const int e = base + static_cast<int>(threadIdx.x);
    if (e < end) stage_entry(a, list, e, &stage[threadIdx.x]);
    __syncthreads();
    for (int k = end - base - 1; k >= 0; --k) {
      const StageEntry& s = stage[k];
      const double q = quad_form(s, cxp, cyp);
      const bool hit = inside && q <= kSupport;
      float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gop = 0.f;
      if (hit) {
        const float rho = __expf(static_cast<float>(-0.5 * q));
        const float raw = s.sigma * rho;
        const float al = fminf(raw, kClamp);
        const double ald = static_cast<double>(al);
        const double om = 1.0 - ald;
        t /= om;  // now T_i = t * pw
        if (t > 0x1p300 && E < 0) {
          t *= 0x1p-600;
          E += kRenorm;
          pw = ldexp(1.0, E);
        }
        const double T = t * pw;
        const double w = ald * T;
        gc0 = static_cast<float>(w * g0);
        gc1 = static_cast<float>(w * g1);
        gc2 = static_cast<float>(w * g2);
        const double c0 = s.c0, c1 = s.c1, c2 = s.c2;
        if (raw < kClamp) {
          const double da = g0 * (c0 - R0) + g1 * (c1 - R1) + g2 * (c2 - R2);
          gop = static_cast<float>(da * T * rho);
        }
        R0 = fma(om, R0, ald * c0);
        R1 = fma(om, R1, ald * c1);
        R2 = fma(om, R2, ald * c2);
      }
      if (__ballot(hit) != 0) {  // wave-uniform: every lane reads the same staged entry
        gc0 = wave_sum(gc0);
        gc1 = wave_sum(gc1);
        gc2 = wave_sum(gc2);
        gop = wave_sum(gop);
        if ((threadIdx.x & 63) == 0) {
          double* acc = a.grad_acc + 4 * static_cast<int64_t>(s.idx);
          unsafeAtomicAdd(acc + 0, static_cast<double>(gc0));
          unsafeAtomicAdd(acc + 1, static_cast<double>(gc1));
          unsafeAtomicAdd(acc + 2, static_cast<double>(gc2));
          unsafeAtomicAdd(acc + 3, static_cast<double>(gop));
        }
      }
    }
  }
}

hipError_t launch_raster(const RasterArgs& a, bool bwd, hipStream_t s) {
  const int64_t n_tiles = static_cast<int64_t>(a.tiles_x) * a.tiles_y;
  const unsigned gt = static_cast<unsigned>((n_tiles + 255) / 256);
  const unsigned gn = static_cast<unsigned>((a.n + 255) / 256);
  if (!bwd) {
    hipLaunchKernelGGL(raster_zero, dim3(gt), dim3(256), 0, s, a.cursor, n_tiles, a.overflow);
    if (a.n > 0) {
      hipLaunchKernelGGL(raster_project, dim3(gn), dim3(256), 0, s, a);
      hipLaunchKernelGGL(raster_bin, dim3(gn), dim3(256), 0, s, a);
    }
    const size_t sm = static_cast<size_t>(a.cap_pow2) * (sizeof(double) + sizeof(int32_t));
    hipLaunchKernelGGL(raster_sort, dim3(static_cast<unsigned>(n_tiles)), dim3(256), sm, s, a);
    hipLaunchKernelGGL(raster_render_fwd, dim3(static_cast<unsigned>(n_tiles)), dim3(256), 0, s,
                       a);
  } else {
    if (a.n == 0) return hipGetLastError();
    hipLaunchKernelGGL(raster_zero_acc, dim3(gn), dim3(256), 0, s, a.grad_acc, a.n);
    hipLaunchKernelGGL(raster_render_bwd, dim3(static_cast<unsigned>(n_tiles)), dim3(256), 0, s,
                       a);
    hipLaunchKernelGGL(raster_finish_grads, dim3(gn), dim3(256), 0, s, a.grad_acc, a.grad_colors,
                       a.grad_opac, a.n);
  }
  return hipGetLastError();
}

}  // namespace nasg
