// Reverse-mode derivative of one quad's substep (everything before the
// in-env pair pass), float32.  Events take the derivative of the branch the
// forward pass took (recorded in Rec); the resting flag carries none.
#pragma once
#include "qs_device.h"

namespace qs {

// Adjoint of the per-quad state (same fields as Quad, resting flag omitted).
struct Adj {
  float x[3], v[3], R[9], w[3], u[4], e[4];
};

__device__ __forceinline__ void cross3f(const float a[3], const float b[3], float o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ __forceinline__ float dot3f(const float a[3], const float b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Physical parameters the adjoint differentiates with respect to.
struct ParAdj {
  float m, jx, jy, jz, t2w;
  float dlag_dtau;  // d a_lag / d tau = -(1 - a_lag) dt / tau^2
};

// l: dL/d(state after the floor step) on entry, dL/d(state at the start of
// the substep) on exit.  gu += dL/d(rotor-speed command uhat);
// gp += dL/d(m, jx, jy, jz, t2w, tau).
__device__ __forceinline__ void quad_vjp(const Consts& c, const QuadPar& p, const ParAdj& pa,
                                         const Rec& r, const float uhat[4], Adj& l,
                                         float gu[4], float gp[6]) {
  const float dt = c.dt;
  // floor hit: z, v, omega were set to constants; R levelled from its heading
  if (r.hit) {
    l.x[2] = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) l.v[k] = l.w[k] = 0.f;
    float g0 = 0.f, g1 = 0.f, g3 = 0.f, g4 = 0.f;
    if (!r.fallback) {
      // column 0 = h = (hx, hy)/nh, column 1 = (-h_y, h_x)
      const float hx = r.hx / r.nh, hy = r.hy / r.nh;
      const float ghx = l.R[0] + l.R[4], ghy = l.R[3] - l.R[1];
      const float dd = ghx * hx + ghy * hy;
      g0 = (ghx - dd * hx) / r.nh;
      g3 = (ghy - dd * hy) / r.nh;
    } else if (r.nk > 0.f) {
      // column 1 = k = (kx, ky)/nk, column 0 = (k_y, -k_x)
      const float kx = r.kx / r.nk, ky = r.ky / r.nk;
      const float gkx = l.R[1] - l.R[3], gky = l.R[4] + l.R[0];
      const float dd = gkx * kx + gky * ky;
      g1 = (gkx - dd * kx) / r.nk;
      g4 = (gky - dd * ky) / r.nk;
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) l.R[k] = 0.f;
    l.R[0] = g0;
    l.R[1] = g1;
    l.R[3] = g3;
    l.R[4] = g4;
  }
  // walls: decay once, then per-axis mirror and clamp (selects: rare events
  // must not split the scheduling region)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    l.v[k] = r.bounced ? l.v[k] * c.col_decay : l.v[k];
    l.v[k] = r.flip[k] ? l.v[k] * -c.e_wall : l.v[k];
    l.x[k] = r.clamp[k] ? 0.f : l.x[k];
  }

  float lT = 0.f, lF[3] = {0.f, 0.f, 0.f}, lt[3] = {0.f, 0.f, 0.f};
  float lm = 0.f, lJ[3] = {0.f, 0.f, 0.f};
  float lP[9], lv0[3], lw0[3];
  const float J[3] = {pa.jx, pa.jy, pa.jz};
  // free flight for every lane; a resting lane (rare) redoes this part below
  {
    // R = Gram-Schmidt(A): c2 = c0 x c1, c1 = b/|b|, b = A1 - (c0.A1) c0, c0 = A0/|A0|
    float lc0[3] = {l.R[0], l.R[3], l.R[6]}, lc1[3] = {l.R[1], l.R[4], l.R[7]};
    const float lc2[3] = {l.R[2], l.R[5], l.R[8]};
    float tmp[3];
    cross3f(r.c1, lc2, tmp);
#pragma unroll
    for (int k = 0; k < 3; ++k) lc0[k] += tmp[k];
    cross3f(lc2, r.c0, tmp);
#pragma unroll
    for (int k = 0; k < 3; ++k) lc1[k] += tmp[k];
    float dd = dot3f(lc1, r.c1);
    float lb[3];
    const float in1 = r.i1;
#pragma unroll
    for (int k = 0; k < 3; ++k) lb[k] = (lc1[k] - dd * r.c1[k]) * in1;
    const float ldp = -dot3f(lb, r.c0);
    float lA1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lA1[k] = fmaf(ldp, r.c0[k], lb[k]);
      lc0[k] += fmaf(-r.dp, lb[k], ldp * r.A1[k]);
    }
    dd = dot3f(lc0, r.c0);
    float lA0[3];
    const float in0 = r.i0;
#pragma unroll
    for (int k = 0; k < 3; ++k) lA0[k] = (lc0[k] - dd * r.c0[k]) * in0;
    // A0 = P0 + dt (P1 w1z - P2 w1y), A1 = P1 + dt (P2 w1x - P0 w1z) (columns)
    const float P0[3] = {r.P[0], r.P[3], r.P[6]}, P1[3] = {r.P[1], r.P[4], r.P[7]},
                P2[3] = {r.P[2], r.P[5], r.P[8]};
    const float lw1[3] = {fmaf(dt, dot3f(P2, lA1), l.w[0]), fmaf(-dt, dot3f(P2, lA0), l.w[1]),
                          fmaf(dt, dot3f(P1, lA0) - dot3f(P0, lA1), l.w[2])};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lP[3 * k + 0] = fmaf(-dt * r.w1[2], lA1[k], lA0[k]);
      lP[3 * k + 1] = fmaf(dt * r.w1[2], lA0[k], lA1[k]);
      lP[3 * k + 2] = dt * (r.w1[0] * lA1[k] - r.w1[1] * lA0[k]);
    }
    // w1 = w0 + dt wdot, wdot_k = (tau_k - (w0 x J w0)_k) / J_k
    float lc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lw0[k] = lw1[k];
      const float lwd = dt * lw1[k];
      const float iJ = k == 0 ? p.ijx : (k == 1 ? p.ijy : p.ijz);
      lt[k] = lwd * iJ;
      lc[k] = -lwd * iJ;
      lJ[k] = -lwd * r.wdot[k] * iJ;
    }
    const float Jw[3] = {J[0] * r.w0[0], J[1] * r.w0[1], J[2] * r.w0[2]};
    cross3f(Jw, lc, tmp);
    float lJw[3];
    cross3f(lc, r.w0, lJw);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      lw0[k] += tmp[k] + J[k] * lJw[k];
      lJ[k] += r.w0[k] * lJw[k];
    }
    // x1 = x0 + dt v1, v1 = v0 + dt acc, acc = F/m - c_d v0/m - g e_z
    const float dm = c.drag * p.inv_m;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float lv1 = fmaf(dt, l.x[k], l.v[k]);
      const float lacc = dt * lv1;
      lv0[k] = fmaf(-dm, lacc, lv1);
      lF[k] = lacc * p.inv_m;
      lm -= (r.F[k] - c.drag * r.v0[k]) * lacc * p.inv_m * p.inv_m;
    }
  }
  if (r.rest) {
    // resting: R held, omega zeroed, v_z zeroed, x_z unchanged
    lm = 0.f;
#pragma unroll
    for (int k = 0; k < 3; ++k) lF[k] = lt[k] = lJ[k] = 0.f;
#pragma unroll
    for (int k = 0; k < 9; ++k) lP[k] = l.R[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) lw0[k] = lv0[k] = 0.f;
    if (!r.guard) {
      const float lv1[2] = {fmaf(dt, l.x[0], l.v[0]), fmaf(dt, l.x[1], l.v[1])};
      const float lfb[2] = {dt * lv1[0] * p.inv_m, dt * lv1[1] * p.inv_m};
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        lv0[k] = lv1[k] * (1.0f - dt * c.drag * p.inv_m);
        lm -= dt * (r.fb[k] - c.drag * r.v0[k]) * lv1[k] * p.inv_m * p.inv_m;
      }
      float lmu = 0.f;
      if (r.statik) {
        if (r.mag > 0.f) {
          const float fx = r.F[0] / r.nf, fy = r.F[1] / r.nf;
          const float dd = lfb[0] * fx + lfb[1] * fy;
          lF[0] += lfb[0] - r.mu_n * (lfb[0] - dd * fx) / r.nf;
          lF[1] += lfb[1] - r.mu_n * (lfb[1] - dd * fy) / r.nf;
          lmu = -dd;
        }
      } else {
        const float vx = r.v0[0] / r.nv, vy = r.v0[1] / r.nv;
        lF[0] += lfb[0];
        lF[1] += lfb[1];
        lmu = -(lfb[0] * vx + lfb[1] * vy);
        const float lvx = -r.mu_n * lfb[0], lvy = -r.mu_n * lfb[1];
        const float dd = lvx * vx + lvy * vy;
        lv0[0] += (lvx - dd * vx) / r.nv;
        lv0[1] += (lvy - dd * vy) / r.nv;
      }
      // mu_n = mu (m g - F_z)
      lm += c.mu * c.g * lmu;
      lF[2] -= c.mu * lmu;
    }
  }
  // F = T * (third column of R)
  lT += lF[0] * r.P[2] + lF[1] * r.P[5] + lF[2] * r.P[8];
  lP[2] = fmaf(r.T, lF[0], lP[2]);
  lP[5] = fmaf(r.T, lF[1], lP[5]);
  lP[8] = fmaf(r.T, lF[2], lP[8]);
  // thrust and torques from the rotor thrusts (X layout FR, BR, BL, FL)
  const float sx[4] = {-1.f, -1.f, 1.f, 1.f}, sy[4] = {-1.f, 1.f, 1.f, -1.f},
              sz[4] = {1.f, -1.f, 1.f, -1.f};
  float lfmax = 0.f, lalag = 0.f;
  const bool noise = (c.flags & F_NOISE) != 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float lf = lT + c.arm_d * (sx[i] * lt[0] + sy[i] * lt[1]) + c.k_tau * sz[i] * lt[2];
    const float lu1 = fmaf(2.0f * p.f_max * r.u1[i], lf, l.u[i]);
    const float le1 = l.e[i] + lf;
    lfmax = fmaf(r.u1[i] * r.u1[i], lf, lfmax);
    // motor noise e1 = a_nd e0 + ns_scale f_max z
    l.e[i] = noise ? c.a_nd * le1 : le1;
    lfmax = noise ? fmaf(c.ns_scale * r.z[i], le1, lfmax) : lfmax;
    // motor lag u1 = u0 + a_lag (uhat - u0)
    l.u[i] = (1.0f - p.a_lag) * lu1;
    gu[i] = fmaf(p.a_lag, lu1, gu[i]);
    lalag = fmaf(uhat[i] - r.u0[i], lu1, lalag);
  }
  // f_max = m g t2w / 4, a_lag = 1 - exp(-dt/tau)
  lm += 0.25f * c.g * pa.t2w * lfmax;
  gp[0] += lm;
  gp[1] += lJ[0];
  gp[2] += lJ[1];
  gp[3] += lJ[2];
  gp[4] += 0.25f * pa.m * c.g * lfmax;
  gp[5] = fmaf(lalag, pa.dlag_dtau, gp[5]);
#pragma unroll
  for (int k = 0; k < 9; ++k) l.R[k] = lP[k];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    l.v[k] = lv0[k];
    l.w[k] = lw0[k];
  }
  // l.x: the start position receives the end position's adjoint unchanged
}

}  // namespace qs
