// The per-primitive skeleton shared by the NASGabor kernel and the other lobe
// families: the ln table, the travelling view slots (set-up, transfer,
// write-out of colours and of the c0 / mean gradients) and the conversion of
// the frame-axis gradients into the stored frame parameters.
//
// Work mapping (both kernels): each primitive owns P consecutive lanes. A view
// chunk of P * VPL views is cut into P view slots; slot j holds views
// v0 + j + P t (t < VPL) with their direction (FP64 and FP32), upstream
// gradient, colour and direction-gradient accumulators. Lane j owns lobe
// lc + j of every P-lobe chunk; P times it evaluates that lobe against the
// slot it holds and passes the slot on to lane j + 1 of the group, so every
// lobe meets every view and every slot ends in its home lane.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

static __constant__ const LogTable kLogTable = make_log_table();

// Copies the ln table into this block's LDS (every thread of the block calls it).
__device__ inline void load_log_table(LogEntry* lds) {
  for (int t = threadIdx.x; t < kLogEntries; t += blockDim.x) lds[t] = kLogTable.e[t];
  __syncthreads();
}

// ------------------------------------------------------ slot transfers
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

// ------------------------------------------------------ view slots
template <int VPL>
struct ViewSlots {
  double dd[VPL][3];      // unit direction, FP64
  float df[VPL][3];       // the same in FP32
  float rinv[VPL];        // 1/|mu - o| (1/|dirs|)
  float gr[VPL][3];       // upstream gradient (0 for a slot beyond V)
  float col[VPL][3];      // colour accumulator
  float gdir[VPL][3];     // dL/dd accumulator
  bool has[VPL];          // the view exists (v < V)
};

// Fills this lane's home slot of the view chunk starting at v0. BC (views
// broadcast): every lane of the group holds the same views v0 + t, t < VPL,
// and only lane 0's colours start from c0 (the group's partial colours are
// summed after the lobes).
template <int P, int VPL, bool BWD, bool BC = false, bool STREAM = false>
__device__ __forceinline__ void slots_setup(const NasgArgs& a, int64_t i, int v0, int j,
                                            const double (&base)[3], const float (&c0)[3],
                                            ViewSlots<VPL>& s) {
  const int64_t N = a.n;
  const int V = a.v;
#pragma unroll
  for (int t = 0; t < VPL; ++t) {
    const int v = BC ? v0 + t : v0 + j + P * t;
    s.has[t] = v < V;
    double e0 = base[0], e1 = base[1], e2 = base[2];
    if (a.dirs == nullptr) {
      const int vc = s.has[t] ? v : 0;
      e0 -= static_cast<double>(a.cams[3 * vc + 0]);
      e1 -= static_cast<double>(a.cams[3 * vc + 1]);
      e2 -= static_cast<double>(a.cams[3 * vc + 2]);
    }
    const double ri = rsqrt64(e0 * e0 + e1 * e1 + e2 * e2);
    s.dd[t][0] = e0 * ri;
    s.dd[t][1] = e1 * ri;
    s.dd[t][2] = e2 * ri;
    s.df[t][0] = static_cast<float>(s.dd[t][0]);
    s.df[t][1] = static_cast<float>(s.dd[t][1]);
    s.df[t][2] = static_cast<float>(s.dd[t][2]);
    s.rinv[t] = static_cast<float>(ri);
    const bool own_c0 = !BC || j == 0;
    s.col[t][0] = own_c0 ? c0[0] : 0.f;
    s.col[t][1] = own_c0 ? c0[1] : 0.f;
    s.col[t][2] = own_c0 ? c0[2] : 0.f;
    s.gdir[t][0] = s.gdir[t][1] = s.gdir[t][2] = 0.f;
    if constexpr (BWD) {
      if (s.has[t]) {
        const int64_t o = (static_cast<int64_t>(v) * N + i) * 3;
        s.gr[t][0] = load_if<STREAM>(&a.grad_rgb[o + 0]);
        s.gr[t][1] = load_if<STREAM>(&a.grad_rgb[o + 1]);
        s.gr[t][2] = load_if<STREAM>(&a.grad_rgb[o + 2]);
      } else {
        s.gr[t][0] = s.gr[t][1] = s.gr[t][2] = 0.f;
      }
    }
  }
}

// Passes slot t on: this lane takes over the slot of lane j + 1.
template <int P, int VPL, bool BWD>
__device__ __forceinline__ void slot_pass(ViewSlots<VPL>& s, int t, int rot_addr) {
  if constexpr (P > 1) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      s.dd[t][c] = group_next<P>(s.dd[t][c], rot_addr);
      s.df[t][c] = group_next<P>(s.df[t][c], rot_addr);
      s.col[t][c] = group_next<P>(s.col[t][c], rot_addr);
      if constexpr (BWD) {
        s.gr[t][c] = group_next<P>(s.gr[t][c], rot_addr);
        s.gdir[t][c] = group_next<P>(s.gdir[t][c], rot_addr);
      }
    }
  }
}

// With the slots home again: the colours of this lane's views, and the c0 and
// mean (or dirs) gradients of the primitive (sums over its views, reduced
// over the lane group, written by lane 0). BC: the group's partial colours
// and direction gradients are first summed over its lanes (each lane then
// holds the totals of all VPL views); lane t % P writes view t's colour, and
// the c0 and mean gradients are not summed over lanes again.
template <int P, int VPL, bool BWD, bool BC = false, bool STREAM = false>
__device__ __forceinline__ void slots_finish(const NasgArgs& a, int64_t i, bool valid, int v0,
                                             int j, bool acc_mode, ViewSlots<VPL>& s) {
  const int64_t N = a.n;
  if constexpr (BC) {
#pragma unroll
    for (int t = 0; t < VPL; ++t) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        s.col[t][c] = group_sum<P>(s.col[t][c]);
        if constexpr (BWD) s.gdir[t][c] = group_sum<P>(s.gdir[t][c]);
      }
    }
  }
  if (a.rgb != nullptr && valid) {
#pragma unroll
    for (int t = 0; t < VPL; ++t) {
      if (!s.has[t] || (BC && j != t % P)) continue;
      const int64_t o = (static_cast<int64_t>(BC ? v0 + t : v0 + j + P * t) * N + i) * 3;
      store_if<STREAM>(s.col[t][0], &a.rgb[o + 0]);
      store_if<STREAM>(s.col[t][1], &a.rgb[o + 1]);
      store_if<STREAM>(s.col[t][2], &a.rgb[o + 2]);
    }
  }
  if constexpr (BWD) {
    float gc0 = 0.f, gc1 = 0.f, gc2 = 0.f, gm0 = 0.f, gm1 = 0.f, gm2 = 0.f;
#pragma unroll
    for (int t = 0; t < VPL; ++t) {
      gc0 += s.gr[t][0];
      gc1 += s.gr[t][1];
      gc2 += s.gr[t][2];
      // d = e/|e|: dL/de = (I - d d^T) dL/dd / |e|
      const float pr =
          s.df[t][0] * s.gdir[t][0] + s.df[t][1] * s.gdir[t][1] + s.df[t][2] * s.gdir[t][2];
      gm0 = fmaf(s.gdir[t][0] - pr * s.df[t][0], s.rinv[t], gm0);
      gm1 = fmaf(s.gdir[t][1] - pr * s.df[t][1], s.rinv[t], gm1);
      gm2 = fmaf(s.gdir[t][2] - pr * s.df[t][2], s.rinv[t], gm2);
    }
    if constexpr (!BC) {
      gc0 = group_sum<P>(gc0);
      gc1 = group_sum<P>(gc1);
      gc2 = group_sum<P>(gc2);
      gm0 = group_sum<P>(gm0);
      gm1 = group_sum<P>(gm1);
      gm2 = group_sum<P>(gm2);
    }
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

// ------------------------------------------------ frame parameter gradients
// (ax, az) = (dL/dx, dL/dz) of one lobe; (xf, zf) its axes in FP32.

// Quaternion frame, f = (q_w, q_x, q_y, q_z) and is = 1/|q|^2. With the unit
// quaternion (w, x, y, z) = q/|q|, the axes are x = (1 - 2(y^2 + z^2),
// 2(xy + wz), 2(xz - wy)) and z = (2(xz + wy), 2(yz - wx), 1 - 2(x^2 + y^2));
// v = J_x^T gx + J_z^T gz with their derivatives in (w, x, y, z), and
// dL/dq = (v - q_hat (q_hat . v)) / |q|. This form has no term larger than
// the gradient's own scale: a lobe that depends on z only, with q near a
// rotation about a coordinate axis, gets small components without cancellation.
__device__ __forceinline__ float4 quat_frame_grad(float fw, float fx, float fy, float fz,
                                                  float fis, const float (&xf)[3],
                                                  const float (&zf)[3], const float (&ax)[3],
                                                  const float (&az)[3]) {
  (void)xf;
  (void)zf;
  const float inv = __builtin_sqrtf(fis);        // 1/|q|
  const float w = fw * inv, x = fx * inv, y = fy * inv, z = fz * inv;
  const float vw = 2.f * (z * ax[1] - y * ax[2] + y * az[0] - x * az[1]);
  const float vx = 2.f * (y * ax[1] + z * ax[2] + z * az[0] - w * az[1]) - 4.f * x * az[2];
  const float vy = 2.f * (x * ax[1] - w * ax[2] + w * az[0] + z * az[1]) - 4.f * y * (ax[0] + az[2]);
  const float vz = 2.f * (w * ax[1] + x * ax[2] + x * az[0] + y * az[1]) - 4.f * z * ax[0];
  const float qv = w * vw + x * vx + y * vy + z * vz;
  float4 gq;
  gq.x = (vw - w * qv) * inv;
  gq.y = (vx - x * qv) * inv;
  gq.z = (vy - y * qv) * inv;
  gq.w = (vz - z * qv) * inv;
  return gq;
}

// The paper's frame (Supplementary C) from raw u with cosines tanh(u) and
// sines sech(u), chained through u (dc/du = s^2, ds/du = -c s), which keeps
// the printed 1/s of Supplementary F's Jacobians out:
//   dx/du_t = s_t (x_1, -x_0, 0),  dz/du_t = s_t (z_1, -z_0, 0),
//   dx/du_p = s_p c_s z,           dz/du_p = -s_p e_p,
//   dx/du_s = s_s (s_s e_p - c_s e_t),
// e_p = (c_t c_p, s_t c_p, -s_p), e_t = (-s_t, c_t, 0).
__device__ __forceinline__ float4 angle_frame_grad(float ct, float st, float cp, float sp,
                                                   float cs, float ss, const float (&xf)[3],
                                                   const float (&zf)[3], const float (&ax)[3],
                                                   const float (&az)[3]) {
  const float ep0 = ct * cp, ep1 = st * cp, ep2 = -sp;
  const float xz = ax[0] * zf[0] + ax[1] * zf[1] + ax[2] * zf[2];
  const float xep = ax[0] * ep0 + ax[1] * ep1 + ax[2] * ep2;
  const float zep = az[0] * ep0 + az[1] * ep1 + az[2] * ep2;
  const float xet = ax[1] * ct - ax[0] * st;
  float4 gq;
  gq.x = st * (ax[0] * xf[1] - ax[1] * xf[0] + az[0] * zf[1] - az[1] * zf[0]);
  gq.y = sp * (cs * xz - zep);
  gq.z = ss * (ss * xep - cs * xet);
  gq.w = 0.f;
  return gq;
}

// Frame of one lobe from its stored frame slot: FP64 axes, and in f the
// values the gradient write-out needs (quaternion and 1/|q|^2, or the paper's
// cosines and sines).
template <bool ANG>
__device__ __forceinline__ void lobe_frame(const float4& q, double (&xa)[3], double (&za)[3],
                                           float (&f)[6]) {
  if constexpr (ANG) {
    // Supplementary C: cosines tanh(u) with sines sqrt(1 - c^2) = sech(u),
    // z = (c_t s_p, s_t s_p, c_p),
    // x = (c_t c_p c_s - s_t s_s, s_t c_p c_s + c_t s_s, -s_p c_s)
    double ct, st, cp, sp, cs, ss;
    tanh_sech(q.x, ct, st);
    tanh_sech(q.y, cp, sp);
    tanh_sech(q.z, cs, ss);
    za[0] = ct * sp;
    za[1] = st * sp;
    za[2] = cp;
    xa[0] = ct * cp * cs - st * ss;
    xa[1] = st * cp * cs + ct * ss;
    xa[2] = -sp * cs;
    f[0] = static_cast<float>(ct);
    f[1] = static_cast<float>(st);
    f[2] = static_cast<float>(cp);
    f[3] = static_cast<float>(sp);
    f[4] = static_cast<float>(cs);
    f[5] = static_cast<float>(ss);
  } else {
    // x = M_x(q)/|q|^2, z = M_z(q)/|q|^2 (homogeneous rotation of q)
    const double qw = q.x, qx = q.y, qy = q.z, qz = q.w;
    const double ww = qw * qw, xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const double is = rcp64(ww + xx + yy + zz);
    xa[0] = (ww + xx - yy - zz) * is;
    xa[1] = 2.0 * (qx * qy + qw * qz) * is;
    xa[2] = 2.0 * (qx * qz - qw * qy) * is;
    za[0] = 2.0 * (qx * qz + qw * qy) * is;
    za[1] = 2.0 * (qy * qz - qw * qx) * is;
    za[2] = (ww - xx - yy + zz) * is;
    f[0] = q.x;
    f[1] = q.y;
    f[2] = q.z;
    f[3] = q.w;
    f[4] = static_cast<float>(is);
    f[5] = 0.f;
  }
}

template <bool ANG>
__device__ __forceinline__ float4 frame_grad(const float (&f)[6], const float (&xf)[3],
                                             const float (&zf)[3], const float (&ax)[3],
                                             const float (&az)[3]) {
  if constexpr (ANG) {
    return angle_frame_grad(f[0], f[1], f[2], f[3], f[4], f[5], xf, zf, ax, az);
  } else {
    return quat_frame_grad(f[0], f[1], f[2], f[3], f[4], xf, zf, ax, az);
  }
}

// Adds or writes a float4 gradient. STREAM: the kernel writes every
// gradient exactly once (one view chunk, no accumulation, so acc_mode is
// false) and its stores cover whole cache lines (one lane per primitive);
// the write is then streaming data. The two forms are chosen at compile time: a run-time
// choice between a plain and a streaming store of the same address would be
// merged by the compiler into one plain store.
template <bool STREAM>
__device__ __forceinline__ void put4(float* base, int64_t li, float4 g, bool acc_mode) {
  float4* dst = reinterpret_cast<float4*>(base) + li;
  if constexpr (STREAM) {
    store_once(f32x4_nt{g.x, g.y, g.z, g.w}, reinterpret_cast<f32x4_nt*>(dst));
  } else {
    if (acc_mode) {
      const float4 o = *dst;
      g.x += o.x;
      g.y += o.y;
      g.z += o.z;
      g.w += o.w;
    }
    *dst = g;
  }
}

// Adds or writes a per-lobe colour-weight gradient in the channel-planar
// layout [K][3][N] (STREAM as for put4). The three old values are loaded
// before any store: N is a run-time stride, so a store to one channel would
// otherwise have to complete before the next channel's load.
template <bool STREAM>
__device__ __forceinline__ void put_rgbw(float* g_rgbw, int lobe, int64_t N, int64_t i, float r0,
                                         float r1, float r2, bool acc_mode) {
  float* dst = g_rgbw + static_cast<int64_t>(lobe) * 3 * N + i;
  if constexpr (STREAM) {
    store_once(r0, dst);
    store_once(r1, dst + N);
    store_once(r2, dst + 2 * N);
  } else {
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

}  // namespace nasg
