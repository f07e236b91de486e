// Boundary-element operator of the direct formulation on top of the FMM
// plans, the FP64 direct sums for the right-hand side and the reaction
// potential, and the FP64 GMRES solver.
//
// Matrix-vector split (Methods, FMM-accelerated evaluation of integral
// operators): A x = P2^T (G - C) P1 x + S x.  P1 turns the P0 coefficients
// into weighted densities at the regular quadrature points, G is the FMM,
// P2^T integrates the FMM output against the test triangles, and S - C (the
// accurate minus the regular-rule values for triangle pairs that share a
// vertex) is precomputed once as a sparse FP64 matrix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fmm_internal.h"

namespace fmm {
int eval_dispatch(fmm_plan *P, const void *q, int nrhs, void *pot, void *grad, hipStream_t s);
}

using fmm::set_error;

namespace {

constexpr double FOUR_PI = 12.566370614359172953850573533118;
constexpr double KCAL = 332.0637;  // e^2/A -> kcal/mol
constexpr int NO = 8;              // outer collapsed Gauss rule, NO x NO points
constexpr int NREM = 4;            // Yukawa remainder rule, NREM x NREM on each triangle

// Gauss-Legendre nodes and weights on [0, 1] (Newton iteration on P_n).
void gauss01(int n, std::vector<double> &x, std::vector<double> &w) {
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p1 = z; p0 = 1; }
      dp = n * (z * p1 - p0) / (z * z - 1);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = 0.5 * (1 - z);
    w[i] = 1.0 / ((1 - z * z) * dp * dp);  // (2/((1-z^2) P'^2)) * 1/2
  }
}

// Collapsed rule on a triangle: barycentric (1 - xi, xi (1 - eta), xi eta),
// weight 2 xi w_i w_j (sums to 1).
void collapsed(int n, std::vector<double> &rule /* 3 per point: l1, l2, w */) {
  std::vector<double> g, w;
  gauss01(n, g, w);
  rule.clear();
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      rule.push_back(g[i] * (1 - g[j]));
      rule.push_back(g[i] * g[j]);
      rule.push_back(2 * g[i] * w[i] * w[j]);
    }
}

void regular(int npts, std::vector<double> &rule) {
  rule.clear();
  if (npts == 3) {
    const double b[3][2] = {{1.0 / 6, 1.0 / 6}, {2.0 / 3, 1.0 / 6}, {1.0 / 6, 2.0 / 3}};
    for (auto &e : b) { rule.push_back(e[0]); rule.push_back(e[1]); rule.push_back(1.0 / 3); }
  } else {
    // degree-4 six-point rule: orbits of (a, a, 1 - 2a)
    const double a1 = 0.445948490915965, w1 = 0.223381589678011;
    const double a2 = 0.091576213509771, w2 = 0.109951743655322;
    const double pts[6][2] = {{a1, 1 - 2 * a1}, {1 - 2 * a1, a1}, {a1, a1}, {a2, 1 - 2 * a2}, {1 - 2 * a2, a2}, {a2, a2}};
    for (int k = 0; k < 6; ++k) {
      rule.push_back(pts[k][0]);
      rule.push_back(pts[k][1]);
      rule.push_back(k < 3 ? w1 : w2);
    }
  }
}

// ---------------------------------------------------------------------------
// device helpers (FP64)
// ---------------------------------------------------------------------------
struct D3 { double x, y, z; };
__device__ inline D3 mk(double a, double b, double c) { return {a, b, c}; }
__device__ inline D3 sub(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ inline D3 add(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ inline D3 scl(D3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ inline D3 cross(D3 a, D3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
__device__ inline double nrm(D3 a) { return sqrt(dot(a, a)); }

// Potential of a uniform unit density on the flat triangle v[3] with unit
// normal n at x (int_T 1/|x - y| dy): a sum over the edges of a logarithm
// term and an arctangent term (the edge-based closed form of the potential
// of a polygon).
__device__ double tri_pot(D3 x, const D3 *v, D3 n) {
  const double d = dot(sub(x, v[0]), n);
  const D3 rho = sub(x, scl(n, d));
  const double ad = fabs(d);
  double out = 0;
  for (int i = 0; i < 3; ++i) {
    const D3 a = v[i], b = v[(i + 1) % 3];
    const D3 e = sub(b, a);
    const double L = nrm(e);
    const D3 lh = scl(e, 1.0 / L);
    const D3 uh = cross(lh, n);
    const double t0 = dot(sub(a, rho), uh);
    const double lp = dot(sub(b, rho), lh), lm = dot(sub(a, rho), lh);
    const double Rp = nrm(sub(x, b)), Rm = nrm(sub(x, a));
    const double R02 = t0 * t0 + d * d;
    if (fabs(t0) > 1e-14 * L) out += t0 * log((Rp + lp) / (Rm + lm));
    out -= ad * (atan2(t0 * lp, R02 + ad * Rp) - atan2(t0 * lm, R02 + ad * Rm));
  }
  return out;
}

// int_T n.(x - y)/|x - y|^3 dy: minus the signed solid angle of the triangle
// seen from x; the principal value 0 for x in the triangle's plane.
__device__ double tri_dlp(D3 x, const D3 *v) {
  const D3 R1 = sub(v[0], x), R2 = sub(v[1], x), R3 = sub(v[2], x);
  const double r1 = nrm(R1), r2 = nrm(R2), r3 = nrm(R3);
  const double num = dot(R1, cross(R2, R3));
  if (fabs(num) <= 1e-13 * r1 * r2 * r3) return 0.0;
  const double den = r1 * r2 * r3 + dot(R1, R2) * r3 + dot(R1, R3) * r2 + dot(R2, R3) * r1;
  return -2.0 * atan2(num, den);
}

// Derivatives of h = (e^{-kappa r} - 1)/(4 pi r), the Yukawa minus the
// Laplace kernel: h'(r); A = h'/r - kappa^2/(8 pi r) (bounded; the
// difference N - x^2/2, N = 1 - (1 + x) e^{-x}, x = kappa r, by its series
// below x = 0.05); B = h'' - h'/r.
__device__ inline void h_derivs(double r, double kappa, double &hp, double &A, double &B) {
  const double x = kappa * r, e = exp(-x);
  const double N = -expm1(-x) - x * e;
  hp = N / (FOUR_PI * r * r);
  const double ser = x * x * x * (-1.0 / 3 + x * (1.0 / 8 + x * (-1.0 / 30 + x * (1.0 / 144 + x * (-1.0 / 840 + x / 5760)))));
  const double Nm = x < 0.05 ? ser : N - 0.5 * x * x;
  A = Nm / (FOUR_PI * r * r * r);
  B = (x * x * e - 3.0 * N) / (FOUR_PI * r * r * r);
}

// -d^2/(dn_x dn_y) of (g_Y - g_L) at u = x - y, r = |u| > 0 (the kernel of
// W_Y - W_L): (nx.ny) h'/r + (u.nx)(u.ny)/r^2 (h'' - h'/r).
__device__ inline double hyper_diff(D3 u, double r, D3 nx, D3 ny, double kappa) {
  double hp, A, B;
  h_derivs(r, kappa, hp, A, B);
  return dot(nx, ny) * hp / r + dot(u, nx) * dot(u, ny) / (r * r) * B;
}

// One thread per singular pair (s, t): D = S - C for V_L, K_L, V_Y, K_Y.
__global__ void k_singular(int64_t npair, const int32_t *__restrict__ ps, const int32_t *__restrict__ pt,
                           const double *__restrict__ tri, const double *__restrict__ normal,
                           const double *__restrict__ area, const double *__restrict__ rule_o, int no,
                           const double *__restrict__ rule_r, int nr, const double *__restrict__ rule_q, int nq,
                           double kappa, double *__restrict__ Dval, double *__restrict__ sdiag, int deriv,
                           double *__restrict__ Dw, double *__restrict__ sdiag_w) {
  const int64_t k = blockIdx.x * 128ll + threadIdx.x;
  if (k >= npair) return;
  const int s = ps[k], t = pt[k];
  D3 vs[3], vt[3];
  for (int i = 0; i < 3; ++i) {
    vs[i] = mk(tri[s * 9 + 3 * i], tri[s * 9 + 3 * i + 1], tri[s * 9 + 3 * i + 2]);
    vt[i] = mk(tri[t * 9 + 3 * i], tri[t * 9 + 3 * i + 1], tri[t * 9 + 3 * i + 2]);
  }
  const D3 nt = mk(normal[t * 3], normal[t * 3 + 1], normal[t * 3 + 2]);
  const double As = area[s], At = area[t];
  auto point = [](const D3 *v, double l1, double l2) {
    return add(add(scl(v[0], 1 - l1 - l2), scl(v[1], l1)), scl(v[2], l2));
  };
  // accurate values: closed-form inner Laplace integrals, outer collapsed rule
  double sv = 0, sk = 0;
  for (int c = 0; c < no; ++c) {
    const D3 x = point(vs, rule_o[3 * c], rule_o[3 * c + 1]);
    const double w = rule_o[3 * c + 2] * As;
    sv += w * tri_pot(x, vt, nt);
    if (s != t) sk += w * tri_dlp(x, vt);  // n.(x - y) = 0 on the element itself
  }
  sv /= FOUR_PI;
  sk /= FOUR_PI;
  double svy = sv, sky = sk;
  if (kappa > 0) {
    for (int a = 0; a < nr; ++a) {
      const D3 x = point(vs, rule_r[3 * a], rule_r[3 * a + 1]);
      const double wa = rule_r[3 * a + 2] * As;
      for (int b = 0; b < nr; ++b) {
        const D3 y = point(vt, rule_r[3 * b], rule_r[3 * b + 1]);
        const double w = wa * rule_r[3 * b + 2] * At;
        const D3 d = sub(x, y);
        const double r = nrm(d);
        const double kr = kappa * r;
        if (r > 0) {
          svy += w * expm1(-kr) / (FOUR_PI * r);
          if (s != t) sky += w * dot(d, nt) * ((1 + kr) * exp(-kr) - 1.0) / (FOUR_PI * r * r * r);
        } else {
          svy += w * (-kappa / FOUR_PI);
        }
      }
    }
  }
  // regular-rule values the quadrature-point sum contains for this pair
  double cv = 0, ck = 0, cvy = 0, cky = 0;
  for (int a = 0; a < nq; ++a) {
    const D3 x = point(vs, rule_q[3 * a], rule_q[3 * a + 1]);
    const double wa = rule_q[3 * a + 2] * As;
    for (int b = 0; b < nq; ++b) {
      const D3 y = point(vt, rule_q[3 * b], rule_q[3 * b + 1]);
      const double w = wa * rule_q[3 * b + 2] * At;
      const D3 d = sub(x, y);
      const double r = nrm(d);
      if (!(r > 0)) continue;
      const double e = exp(-kappa * r);
      const double dn = dot(d, nt);
      cv += w / (FOUR_PI * r);
      ck += w * dn / (FOUR_PI * r * r * r);
      cvy += w * e / (FOUR_PI * r);
      cky += w * dn * (1 + kappa * r) * e / (FOUR_PI * r * r * r);
    }
  }
  Dval[4 * k + 0] = sv - cv;
  Dval[4 * k + 1] = sk - ck;
  Dval[4 * k + 2] = svy - cvy;
  Dval[4 * k + 3] = sky - cky;
  if (s == t) {
    sdiag[2 * s] = sv;
    sdiag[2 * s + 1] = svy;
  }
  if (!deriv) return;
  // W_Y - W_L: its 1/r part (kappa^2/2)(ns.nt)/(4 pi r) through the Laplace
  // single-layer value above, the rest on the remainder rule; minus the
  // regular-rule value
  const D3 ns = mk(normal[s * 3], normal[s * 3 + 1], normal[s * 3 + 2]);
  const double nn = dot(ns, nt);
  double ws = 0.5 * kappa * kappa * nn * sv;
  for (int a = 0; a < nr; ++a) {
    const D3 x = point(vs, rule_r[3 * a], rule_r[3 * a + 1]);
    const double wa = rule_r[3 * a + 2] * As;
    for (int b = 0; b < nr; ++b) {
      const D3 y = point(vt, rule_r[3 * b], rule_r[3 * b + 1]);
      const double w = wa * rule_r[3 * b + 2] * At;
      const D3 d = sub(x, y);
      const double r = nrm(d);
      if (r > 0) {
        double hp, A, B;
        h_derivs(r, kappa, hp, A, B);
        ws += w * (nn * A + dot(d, ns) * dot(d, nt) / (r * r) * B);
      } else {
        ws += w * (-nn * kappa * kappa * kappa / (12.0 * M_PI));
      }
    }
  }
  double wc = 0;
  for (int a = 0; a < nq; ++a) {
    const D3 x = point(vs, rule_q[3 * a], rule_q[3 * a + 1]);
    const double wa = rule_q[3 * a + 2] * As;
    for (int b = 0; b < nq; ++b) {
      const D3 y = point(vt, rule_q[3 * b], rule_q[3 * b + 1]);
      const D3 d = sub(x, y);
      const double r = nrm(d);
      if (r > 0) wc += wa * rule_q[3 * b + 2] * At * hyper_diff(d, r, ns, nt, kappa);
    }
  }
  Dw[k] = ws - wc;
  if (s == t) sdiag_w[s] = ws;
}

// Coefficients of the two derivative formulations.  The monopole + dipole
// FMM pass returns pot_L = K_L u + sL V_L v and pot_Y = K_Y u + sY V_Y v (charge
// scales sL, sY) with their gradients; the rows are then
//   y1 = d1 A u + c1L pot_L - c1Y pot_Y
//   y2 = d2 A v + c2 n.(grad pot_L - grad pot_Y)
// since n.grad pot = -W u + s K' v.  With e21 = eps2/eps1, e12 = eps1/eps2:
//   interior (eq:juffer): sL = -1,   sY = -e12, d1 = (1 + e21)/2, c1L = 1,   c1Y = e21, d2 = (1 + e12)/2, c2 = 1
//   exterior (eq:lu):     sL = -e21, sY = -1,   d1 = (1 + e12)/2, c1L = e12, c1Y = 1,   d2 = (1 + e12)/2, c2 = e12
struct DerivCoef {
  double sL, sY, d1, c1L, c1Y, d2, c2;
};

DerivCoef deriv_coef(int formulation, double eps_in, double eps_out) {
  const double e21 = eps_out / eps_in, e12 = eps_in / eps_out;
  if (formulation == FMM_BEM_EXTERIOR || formulation == FMM_BEM_EXTERIOR_P1)
    return {-e21, -1.0, 0.5 * (1 + e12), e12, 1.0, 0.5 * (1 + e12), e12};
  return {-1.0, -e12, 0.5 * (1 + e21), 1.0, e21, 0.5 * (1 + e12), 1.0};
}

// ---------------------------------------------------------------------------
// P1 (continuous piecewise-linear) elements: hat function of vertex i is the
// barycentric coordinate lambda_a of the corner a with tri[a] = i
// ---------------------------------------------------------------------------

// In-plane moments of the flat triangle v[3] (unit normal n) seen from x,
// with d = n.(x - v0), rho = x - d n, R = |x - y|:
//   G  = int_T (y - rho)/R dy,   dH = d int_T (y - rho)/R^3 dy.
// (y - rho)/R is the in-plane gradient of R and (y - rho)/R^3 that of -1/R,
// so by the divergence theorem in the plane each is a sum over the edges of
// the outward edge normal m times int_e R dl = (l R + c^2 log(l + R))/2,
// resp. -int_e dl/R = -log(l + R), between the edge's end coordinates
// (R^2 = l^2 + c^2 along the edge).  With them a linear density lambda has
//   int_T lambda/R = lambda(rho) P + grad lambda . G,
//   int_T lambda d/R^3 = lambda(rho) D + grad lambda . dH
// (P, D the uniform-density values of tri_pot and tri_dlp).
__device__ void tri_lin_moments(D3 x, const D3 *v, D3 n, D3 &G, D3 &dH) {
  const double d = dot(sub(x, v[0]), n);
  const D3 rho = sub(x, scl(n, d));
  G = mk(0, 0, 0);
  dH = mk(0, 0, 0);
  for (int i = 0; i < 3; ++i) {
    const D3 a = v[i], b = v[(i + 1) % 3];
    const D3 e = sub(b, a);
    const double L = nrm(e);
    const D3 lh = scl(e, 1.0 / L);
    const D3 m = cross(lh, n);
    const double t0 = dot(sub(a, rho), m);
    const double lp = dot(sub(b, rho), lh), lm = dot(sub(a, rho), lh);
    const double Rp = nrm(sub(x, b)), Rm = nrm(sub(x, a));
    const double c2 = t0 * t0 + d * d;
    double lg = 0;  // log((lp + Rp)/(lm + Rm)); l + R = c^2/(R - l) for l < 0
    if (c2 > 1e-28 * L * L) {
      if (lm >= 0) lg = log((lp + Rp) / (lm + Rm));
      else if (lp <= 0) lg = log((Rm - lm) / (Rp - lp));
      else lg = log((lp + Rp) * (Rm - lm) / c2);
    }
    G = add(G, scl(m, 0.5 * (lp * Rp - lm * Rm + c2 * lg)));
    dH = sub(dH, scl(m, d * lg));
  }
}

// One thread per singular pair (s, t): the 3 x 3 blocks [corner of s][corner
// of t] of S - C for V_L, K_L, V_Y, K_Y and W_Y - W_L with hat-function
// weights.  S: the Laplace inner integral in closed form for the linear
// density on t, the outer integral on the collapsed rule; the bounded
// Yukawa-minus-Laplace remainders (and the non-1/r part of W_Y - W_L) on
// the collapsed rule on both triangles.  C: the regular rule, zero-distance
// point pairs left out.  Computed in FP64 and stored pair-minor as SV (FP32
// for single-precision operators, whose quadrature-point sums are FP32
// anyway): B[(9 op + 3 a + b) * npair + k], 45 arrays of npair values, so
// that consecutive pairs read consecutive addresses.
template <typename SV>
__global__ __launch_bounds__(128) void k_singular_p1(int64_t npair, const int32_t *__restrict__ ps,
                                                     const int32_t *__restrict__ pt, const double *__restrict__ tri,
                                                     const double *__restrict__ normal,
                                                     const double *__restrict__ area,
                                                     const double *__restrict__ rule_o, int no,
                                                     const double *__restrict__ rule_r, int nr,
                                                     const double *__restrict__ rule_q, int nq, double kappa,
                                                     SV *__restrict__ B) {
  const int64_t k = blockIdx.x * 128ll + threadIdx.x;
  if (k >= npair) return;
  const int s = ps[k], t = pt[k];
  D3 vs[3], vt[3];
  for (int i = 0; i < 3; ++i) {
    vs[i] = mk(tri[s * 9 + 3 * i], tri[s * 9 + 3 * i + 1], tri[s * 9 + 3 * i + 2]);
    vt[i] = mk(tri[t * 9 + 3 * i], tri[t * 9 + 3 * i + 1], tri[t * 9 + 3 * i + 2]);
  }
  const D3 nt = mk(normal[t * 3], normal[t * 3 + 1], normal[t * 3 + 2]);
  const D3 ns = mk(normal[s * 3], normal[s * 3 + 1], normal[s * 3 + 2]);
  const double As = area[s], At = area[t], nn = dot(ns, nt);
  const bool same = s == t;
  D3 gt[3];  // gradients of t's hat functions
  for (int b = 0; b < 3; ++b) gt[b] = scl(cross(nt, sub(vt[(b + 2) % 3], vt[(b + 1) % 3])), 0.5 / At);
  auto point = [](const D3 *v, double l1, double l2) {
    return add(add(scl(v[0], 1 - l1 - l2), scl(v[1], l1)), scl(v[2], l2));
  };
  double VL[9], KL[9], VY[9], KY[9], W[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) VL[i] = KL[i] = 0;
  for (int c = 0; c < no; ++c) {
    const double l1 = rule_o[3 * c], l2 = rule_o[3 * c + 1];
    const D3 x = point(vs, l1, l2);
    const double w = rule_o[3 * c + 2] * As;
    const double la[3] = {1 - l1 - l2, l1, l2};
    const double P = tri_pot(x, vt, nt);
    const double D = same ? 0.0 : tri_dlp(x, vt);
    D3 G, dH;
    tri_lin_moments(x, vt, nt, G, dH);
    const D3 rho = sub(x, scl(nt, dot(sub(x, vt[0]), nt)));
    const D3 rr = sub(rho, vt[0]);
    double iv[3], ik[3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const double lr = (b == 0 ? 1.0 : 0.0) + dot(gt[b], rr);
      iv[b] = lr * P + dot(gt[b], G);
      ik[b] = lr * D + dot(gt[b], dH);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        VL[3 * a + b] += w * la[a] * iv[b];
        KL[3 * a + b] += w * la[a] * ik[b];
      }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    VL[i] /= FOUR_PI;
    KL[i] = same ? 0.0 : KL[i] / FOUR_PI;
    VY[i] = VL[i];
    KY[i] = KL[i];
    W[i] = 0.5 * kappa * kappa * nn * VL[i];  // the 1/r part of W_Y - W_L
  }
  for (int a = 0; a < nr; ++a) {
    const double l1 = rule_r[3 * a], l2 = rule_r[3 * a + 1];
    const D3 x = point(vs, l1, l2);
    const double wa = rule_r[3 * a + 2] * As;
    const double la[3] = {1 - l1 - l2, l1, l2};
    for (int b = 0; b < nr; ++b) {
      const double m1 = rule_r[3 * b], m2 = rule_r[3 * b + 1];
      const D3 y = point(vt, m1, m2);
      const double w = wa * rule_r[3 * b + 2] * At;
      const double lb[3] = {1 - m1 - m2, m1, m2};
      const D3 d = sub(x, y);
      const double r = nrm(d);
      double rv, rk = 0, rw;
      if (r > 0) {
        const double kr = kappa * r;
        rv = expm1(-kr) / (FOUR_PI * r);
        if (!same) rk = dot(d, nt) * ((1 + kr) * exp(-kr) - 1.0) / (FOUR_PI * r * r * r);
        double hp, A, Bh;
        h_derivs(r, kappa, hp, A, Bh);
        rw = nn * A + dot(d, ns) * dot(d, nt) / (r * r) * Bh;
      } else {
        rv = -kappa / FOUR_PI;
        rw = -nn * kappa * kappa * kappa / (12.0 * M_PI);
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double ww = w * la[i] * lb[j];
          VY[3 * i + j] += ww * rv;
          KY[3 * i + j] += ww * rk;
          W[3 * i + j] += ww * rw;
        }
    }
  }
  // minus the regular-rule values the quadrature-point sums contain
  for (int a = 0; a < nq; ++a) {
    const double l1 = rule_q[3 * a], l2 = rule_q[3 * a + 1];
    const D3 x = point(vs, l1, l2);
    const double wa = rule_q[3 * a + 2] * As;
    const double la[3] = {1 - l1 - l2, l1, l2};
    for (int b = 0; b < nq; ++b) {
      const double m1 = rule_q[3 * b], m2 = rule_q[3 * b + 1];
      const D3 y = point(vt, m1, m2);
      const D3 d = sub(x, y);
      const double r = nrm(d);
      if (!(r > 0)) continue;
      const double w = wa * rule_q[3 * b + 2] * At;
      const double lb[3] = {1 - m1 - m2, m1, m2};
      const double e = exp(-kappa * r), dn = dot(d, nt);
      const double gl = 1.0 / (FOUR_PI * r), kl = dn / (FOUR_PI * r * r * r);
      const double gy = e * gl, ky = (1 + kappa * r) * e * kl, hw = hyper_diff(d, r, ns, nt, kappa);
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double ww = w * la[i] * lb[j];
          VL[3 * i + j] -= ww * gl;
          KL[3 * i + j] -= ww * kl;
          VY[3 * i + j] -= ww * gy;
          KY[3 * i + j] -= ww * ky;
          W[3 * i + j] -= ww * hw;
        }
    }
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    B[(0 + i) * npair + k] = (SV)VL[i];
    B[(9 + i) * npair + k] = (SV)KL[i];
    B[(18 + i) * npair + k] = (SV)VY[i];
    B[(27 + i) * npair + k] = (SV)KY[i];
    B[(36 + i) * npair + k] = (SV)W[i];
  }
}

// The K' blocks of every pair (s, t) from the transposed pair's K blocks,
// KT[(9 kern + 3 a + b) * npair + k] = K_kern[t, s][b][a] (kern 0: Laplace,
// 1: Yukawa), pair-minor like B.
template <typename SV>
__global__ void k_p1_transpose(int64_t npair, const int32_t *__restrict__ tr, const SV *__restrict__ B,
                               SV *__restrict__ KT) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= npair) return;
  const int64_t kt = tr[k];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      KT[(3 * a + b) * npair + k] = B[(9 + 3 * b + a) * npair + kt];
      KT[(9 + 3 * a + b) * npair + k] = B[(27 + 3 * b + a) * npair + kt];
    }
}

// One thread per singular pair (s, t): the S - C terms of both rows for the
// three corners of s, from t's vertex values:
//   P[a]     = sum_b c1L (K_L u_b + sL V_L v_b) - c1Y (K_Y u_b + sY V_Y v_b)
//   P[3 + a] = sum_b (W_Y - W_L) u_b + sL K'_L v_b - sY K'_Y v_b
// (pair-minor, P[j * npair + k]); k_p1_corner adds them per triangle.
template <typename SV>
__global__ void k_p1_pairs(int64_t npair, const int32_t *__restrict__ pt, const int32_t *__restrict__ tris,
                           const SV *__restrict__ B, const SV *__restrict__ KT, const double *__restrict__ x,
                           int64_t nv, DerivCoef c, double *__restrict__ P) {
  const int64_t k = blockIdx.x * 256ll + threadIdx.x;
  if (k >= npair) return;
  const int t = pt[k];
  double u[3], v[3];
  for (int b = 0; b < 3; ++b) {
    const int32_t vb = tris[3 * t + b];
    u[b] = x[vb];
    v[b] = x[nv + vb];
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double p1 = 0, p2 = 0;
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const int ab = 3 * a + b;
      const double vl = (double)B[ab * npair + k], kl = (double)B[(9 + ab) * npair + k];
      const double vy = (double)B[(18 + ab) * npair + k], ky = (double)B[(27 + ab) * npair + k];
      const double w = (double)B[(36 + ab) * npair + k];
      const double ktl = (double)KT[ab * npair + k], kty = (double)KT[(9 + ab) * npair + k];
      p1 += c.c1L * (kl * u[b] + c.sL * vl * v[b]) - c.c1Y * (ky * u[b] + c.sY * vy * v[b]);
      p2 += w * u[b] + c.sL * ktl * v[b] - c.sY * kty * v[b];
    }
    P[a * npair + k] = p1;
    P[(3 + a) * npair + k] = p2;
  }
}

// P1 sources at quadrature point i of triangle t: the vertex values
// interpolated, u(x_i) = sum_a lambda_a(xi_i) u[tri_a]; charge W_i vscale
// v(x_i), dipole W_i u(x_i) n_t.
template <typename T>
__global__ void k_p1_src(int64_t nt, int nq, const int32_t *__restrict__ tris, const double *__restrict__ rule_q,
                         const double *__restrict__ x, int64_t nv, double vscale, const double *__restrict__ qw,
                         const double *__restrict__ normal, T *__restrict__ q, T *__restrict__ dip) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= nt * nq) return;
  const int64_t t = i / nq;
  const int a = (int)(i - t * nq);
  const double l1 = rule_q[3 * a], l2 = rule_q[3 * a + 1];
  const double la[3] = {1 - l1 - l2, l1, l2};
  double u = 0, v = 0;
  for (int c = 0; c < 3; ++c) {
    const int32_t vi = tris[3 * t + c];
    u += la[c] * x[vi];
    v += la[c] * x[nv + vi];
  }
  const double w = qw[i];
  q[i] = (T)(w * vscale * v);
  dip[3 * i + 0] = (T)(w * u * normal[3 * t + 0]);
  dip[3 * i + 1] = (T)(w * u * normal[3 * t + 1]);
  dip[3 * i + 2] = (T)(w * u * normal[3 * t + 2]);
}

// Exterior formulation on P1 elements, per triangle s and corner a (the
// test function lambda_a on s): the quadrature-point fields weighted by
// W_j lambda_a(xi_j), the S - C terms of s's singular pairs (k_p1_pairs, in
// pair order), and s's part of the mass matrix
// (A/12 (1 + delta_ab)); cb[s][a][0..1] for the two rows, added into the
// vertices by k_p1_gather.  Coefficients as k_bem_p2_deriv.
template <typename T>
__global__ __launch_bounds__(64) void k_p1_corner(int64_t nt, int nq, const T *__restrict__ potl,
                                                  const T *__restrict__ gradl, const T *__restrict__ poty,
                                                  const T *__restrict__ grady, const double *__restrict__ qw,
                                                  const double *__restrict__ rule_q, const double *__restrict__ area,
                                                  const double *__restrict__ normal, const int32_t *__restrict__ tris,
                                                  const int32_t *__restrict__ sp_off, int64_t npair,
                                                  const double *__restrict__ P, const double *__restrict__ x,
                                                  int64_t nv, DerivCoef c, double *__restrict__ cb) {
  // one wave per 64 consecutive triangles; their pairs are one contiguous
  // range, staged through LDS 256 pairs at a time with coalesced loads, each
  // lane adding its own pairs in ascending order
  __shared__ double sP[6][256];
  const int64_t s0 = (int64_t)blockIdx.x * 64, s = s0 + threadIdx.x;
  const bool act = s < nt;
  const int k_lo = sp_off[s0], k_hi = sp_off[min(nt, s0 + 64)];
  const int my0 = act ? sp_off[s] : 0, my1 = act ? sp_off[s + 1] : 0;
  double b1[3] = {0, 0, 0}, b2[3] = {0, 0, 0};
  for (int c0 = k_lo; c0 < k_hi; c0 += 256) {
    const int c1 = min(k_hi, c0 + 256);
    for (int i = threadIdx.x; i < c1 - c0; i += 64)
      for (int j = 0; j < 6; ++j) sP[j][i] = P[j * npair + c0 + i];
    __syncthreads();
    for (int k = max(my0, c0); k < min(my1, c1); ++k)
      for (int a = 0; a < 3; ++a) {
        b1[a] += sP[a][k - c0];
        b2[a] += sP[3 + a][k - c0];
      }
    __syncthreads();
  }
  if (!act) return;
  const double n0 = normal[3 * s], n1 = normal[3 * s + 1], n2 = normal[3 * s + 2];
  double r1[3] = {0, 0, 0}, r2[3] = {0, 0, 0};
  for (int j = 0; j < nq; ++j) {
    const int64_t i = s * nq + j;
    const double l1 = rule_q[3 * j], l2 = rule_q[3 * j + 1];
    const double la[3] = {1 - l1 - l2, l1, l2};
    const double f1 = qw[i] * (c.c1L * (double)potl[i] - c.c1Y * (double)poty[i]);
    const double f2 = qw[i] * (n0 * ((double)gradl[3 * i] - (double)grady[3 * i]) +
                               n1 * ((double)gradl[3 * i + 1] - (double)grady[3 * i + 1]) +
                               n2 * ((double)gradl[3 * i + 2] - (double)grady[3 * i + 2]));
    for (int a = 0; a < 3; ++a) {
      r1[a] += la[a] * f1;
      r2[a] += la[a] * f2;
    }
  }
  double us = 0, vs = 0, ua[3], va[3];
  for (int a = 0; a < 3; ++a) {
    const int32_t vi = tris[3 * s + a];
    ua[a] = x[vi];
    va[a] = x[nv + vi];
    us += ua[a];
    vs += va[a];
  }
  const double m = area[s] / 12.0;
  for (int a = 0; a < 3; ++a) {
    cb[(s * 3 + a) * 2 + 0] = c.d1 * m * (ua[a] + us) + r1[a] + b1[a];
    cb[(s * 3 + a) * 2 + 1] = c.d2 * m * (va[a] + vs) + c.c2 * (r2[a] + b2[a]);
  }
}

// cb[s][a][col] = sum_j W_j lambda_a(xi_j) f_j (a field tested with the hat
// functions, per triangle corner).
__global__ void k_p1_project(int64_t nt, int nq, const double *__restrict__ qw, const double *__restrict__ rule_q,
                             const double *__restrict__ f, int col, double *__restrict__ cb) {
  const int64_t s = blockIdx.x * 256ll + threadIdx.x;
  if (s >= nt) return;
  double r[3] = {0, 0, 0};
  for (int j = 0; j < nq; ++j) {
    const double l1 = rule_q[3 * j], l2 = rule_q[3 * j + 1];
    const double wf = qw[s * nq + j] * f[s * nq + j];
    r[0] += (1 - l1 - l2) * wf;
    r[1] += l1 * wf;
    r[2] += l2 * wf;
  }
  for (int a = 0; a < 3; ++a) cb[(s * 3 + a) * 2 + col] = r[a];
}

// y[i] = sum over the corners (s, a) at vertex i (ascending s) of cb[s][a][0],
// y[nv + i] the same of cb[s][a][1]: a fixed order, so results do not depend
// on scheduling.
__global__ void k_p1_gather(int64_t nv, const int32_t *__restrict__ vt_off, const int32_t *__restrict__ vt_list,
                            const double *__restrict__ cb, double *__restrict__ y) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= nv) return;
  double a0 = 0, a1 = 0;
  for (int k = vt_off[i]; k < vt_off[i + 1]; ++k) {
    const int32_t c = vt_list[k];
    a0 += cb[2 * (int64_t)c];
    a1 += cb[2 * (int64_t)c + 1];
  }
  y[i] = a0;
  y[nv + i] = a1;
}

// Lumped mass preconditioner on P1 elements: per vertex diag(1/Ml, 1/Ml),
// Ml = sum over the triangles at the vertex of area/3 (the mass matrix's row
// sum); stored as 2 x 2 blocks for k_precond_apply.
__global__ void k_precond_setup_lumped(int64_t nv, const int32_t *__restrict__ vt_off,
                                       const int32_t *__restrict__ vt_list, const double *__restrict__ area,
                                       double *__restrict__ pre) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= nv) return;
  double ml = 0;
  for (int k = vt_off[i]; k < vt_off[i + 1]; ++k) ml += area[vt_list[k] / 3] / 3.0;
  pre[4 * i + 0] = 1.0 / ml;
  pre[4 * i + 1] = 0.0;
  pre[4 * i + 2] = 0.0;
  pre[4 * i + 3] = 1.0 / ml;
}

// Inverse of the 2x2 diagonal block of a derivative formulation,
// [[d1 A, c1L sL V_L,ss - c1Y sY V_Y,ss], [c2 (W_Y - W_L)_ss, d2 A]]
// (K_ss = K'_ss = 0 on a flat triangle).
__global__ void k_precond_setup_deriv(int64_t nt, const double *__restrict__ area, const double *__restrict__ sdiag,
                                      const double *__restrict__ sdiag_w, DerivCoef c, double *__restrict__ pre) {
  const int64_t s = blockIdx.x * 256ll + threadIdx.x;
  if (s >= nt) return;
  const double a = c.d1 * area[s], b = c.c1L * c.sL * sdiag[2 * s] - c.c1Y * c.sY * sdiag[2 * s + 1],
               cw = c.c2 * sdiag_w[s], d = c.d2 * area[s];
  const double det = a * d - b * cw;
  pre[4 * s + 0] = d / det;
  pre[4 * s + 1] = -b / det;
  pre[4 * s + 2] = -cw / det;
  pre[4 * s + 3] = a / det;
}

// Mass-matrix preconditioner: P = diag(M, M), M = diag(areas) (the Galerkin
// mass matrix of P0 elements is diagonal, so mass lumping is exact).
__global__ void k_precond_setup_mass(int64_t nt, const double *__restrict__ area, double *__restrict__ pre) {
  const int64_t s = blockIdx.x * 256ll + threadIdx.x;
  if (s >= nt) return;
  pre[4 * s + 0] = 1.0 / area[s];
  pre[4 * s + 1] = 0.0;
  pre[4 * s + 2] = 0.0;
  pre[4 * s + 3] = 1.0 / area[s];
}

// Inverse of the 2x2 diagonal block [[A/2, -V_L,ss], [A/2, (e1/e2) V_Y,ss]]
// (K_ss = 0 on a flat triangle).
__global__ void k_precond_setup(int64_t nt, const double *__restrict__ area, const double *__restrict__ sdiag,
                                double eratio, double *__restrict__ pre) {
  const int64_t s = blockIdx.x * 256ll + threadIdx.x;
  if (s >= nt) return;
  const double a = 0.5 * area[s], b = -sdiag[2 * s], c = 0.5 * area[s], d = eratio * sdiag[2 * s + 1];
  const double det = a * d - b * c;
  pre[4 * s + 0] = d / det;
  pre[4 * s + 1] = -b / det;
  pre[4 * s + 2] = -c / det;
  pre[4 * s + 3] = a / det;
}

__global__ void k_precond_apply(int64_t nt, const double *__restrict__ pre, const double *__restrict__ x,
                                double *__restrict__ y) {
  const int64_t s = blockIdx.x * 256ll + threadIdx.x;
  if (s >= nt) return;
  const double u = x[s], v = x[nt + s];
  y[s] = pre[4 * s] * u + pre[4 * s + 1] * v;
  y[nt + s] = pre[4 * s + 2] * u + pre[4 * s + 3] * v;
}

// P1 for the monopole + dipole evaluation: at quadrature point i of triangle
// t, charge W_i v_t (single layer) and dipole W_i u_t n_t (double layer).
template <typename T>
__global__ void k_bem_p1_md(int64_t nt, int nq, const double *__restrict__ x, const double *__restrict__ qw,
                            const double *__restrict__ normal, T *__restrict__ q, T *__restrict__ dip) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= nt * nq) return;
  const int64_t t = i / nq;
  const double w = qw[i], u = x[t], v = x[nt + t];
  q[i] = (T)(w * v);
  dip[3 * i + 0] = (T)(w * u * normal[3 * t + 0]);
  dip[3 * i + 1] = (T)(w * u * normal[3 * t + 1]);
  dip[3 * i + 2] = (T)(w * u * normal[3 * t + 2]);
}

// P2^T and assembly for the monopole + dipole evaluation: the FMM returned,
// per quadrature point, pot_L = K_L u - V_L v and pot_Y = K_Y u - (eps_in /
// eps_out) V_Y v (regular parts), so
//   y1 = M u / 2 + P2^T pot_L + (S - C) terms,  y2 = M u / 2 - P2^T pot_Y + (S - C) terms.
template <typename T>
__global__ __launch_bounds__(64) void k_bem_p2_md(int64_t nt, int nq, const T *__restrict__ potl,
                                                  const T *__restrict__ poty, const double *__restrict__ qw,
                                                  const double *__restrict__ area, const int32_t *__restrict__ sp_off,
                                                  const int32_t *__restrict__ sp_idx, const double *__restrict__ Dval,
                                                  const double *__restrict__ x, double eratio,
                                                  double *__restrict__ y) {
  // one wave per 64 consecutive triangles: their singular pairs are one
  // contiguous range, staged through LDS 256 pairs at a time with coalesced
  // loads; each lane adds its own pairs in ascending order
  __shared__ double sD[256 * 4];
  __shared__ int32_t sT[256];
  const int64_t s0 = (int64_t)blockIdx.x * 64, s = s0 + threadIdx.x;
  const bool act = s < nt;
  const int k_lo = sp_off[s0], k_hi = sp_off[min(nt, s0 + 64)];
  const int my0 = act ? sp_off[s] : 0, my1 = act ? sp_off[s + 1] : 0;
  double al = 0, ay = 0;
  if (act)
    for (int a = 0; a < nq; ++a) {
      const int64_t i = s * nq + a;
      al += qw[i] * (double)potl[i];
      ay += qw[i] * (double)poty[i];
    }
  for (int c0 = k_lo; c0 < k_hi; c0 += 256) {
    const int c1 = min(k_hi, c0 + 256);
    for (int i = threadIdx.x; i < 4 * (c1 - c0); i += 64) sD[i] = Dval[4 * (int64_t)c0 + i];
    for (int i = threadIdx.x; i < c1 - c0; i += 64) sT[i] = sp_idx[c0 + i];
    __syncthreads();
    for (int k = max(my0, c0); k < min(my1, c1); ++k) {
      const int t = sT[k - c0];
      const double *D = sD + 4 * (k - c0);
      const double u = x[t], v = x[nt + t];
      al += D[1] * u - D[0] * v;
      ay += D[3] * u - eratio * D[2] * v;
    }
    __syncthreads();
  }
  if (!act) return;
  const double hu = 0.5 * area[s] * x[s];
  y[s] = hu + al;
  y[nt + s] = hu - ay;
}

// P2^T and assembly for the derivative formulations (coefficients in
// DerivCoef), regular parts from the FMM plus the S - C terms; the K'
// corrections are those of K on the transposed pair.
template <typename T>
__global__ __launch_bounds__(64) void k_bem_p2_deriv(
    int64_t nt, int nq, const T *__restrict__ potl, const T *__restrict__ gradl, const T *__restrict__ poty,
    const T *__restrict__ grady, const double *__restrict__ qw, const double *__restrict__ area,
    const double *__restrict__ normal, const int32_t *__restrict__ sp_off, const int32_t *__restrict__ sp_idx,
    const int32_t *__restrict__ sp_tr, const double *__restrict__ Dval, const double *__restrict__ Dw,
    const double *__restrict__ x, DerivCoef c, double *__restrict__ y) {
  // staging as in k_bem_p2_md; the loading lanes also fetch the transposed
  // pairs' K values
  __shared__ double sD[256 * 4], sW[256], sKt[256 * 2];
  __shared__ int32_t sT[256];
  const int64_t s0 = (int64_t)blockIdx.x * 64, s = s0 + threadIdx.x;
  const bool act = s < nt;
  const int k_lo = sp_off[s0], k_hi = sp_off[min(nt, s0 + 64)];
  const int my0 = act ? sp_off[s] : 0, my1 = act ? sp_off[s + 1] : 0;
  double a1 = 0, a2 = 0;
  if (act) {
    const double n0 = normal[3 * s], n1 = normal[3 * s + 1], n2 = normal[3 * s + 2];
    for (int a = 0; a < nq; ++a) {
      const int64_t i = s * nq + a;
      a1 += qw[i] * (c.c1L * (double)potl[i] - c.c1Y * (double)poty[i]);
      a2 += qw[i] * (n0 * ((double)gradl[3 * i] - (double)grady[3 * i]) +
                     n1 * ((double)gradl[3 * i + 1] - (double)grady[3 * i + 1]) +
                     n2 * ((double)gradl[3 * i + 2] - (double)grady[3 * i + 2]));
    }
  }
  double b1 = 0, b2 = 0;
  for (int c0 = k_lo; c0 < k_hi; c0 += 256) {
    const int c1 = min(k_hi, c0 + 256);
    for (int i = threadIdx.x; i < 4 * (c1 - c0); i += 64) sD[i] = Dval[4 * (int64_t)c0 + i];
    for (int i = threadIdx.x; i < c1 - c0; i += 64) {
      const int k = c0 + i, kt = sp_tr[k];
      sT[i] = sp_idx[k];
      sW[i] = Dw[k];
      sKt[2 * i] = Dval[4 * (int64_t)kt + 1];
      sKt[2 * i + 1] = Dval[4 * (int64_t)kt + 3];
    }
    __syncthreads();
    for (int k = max(my0, c0); k < min(my1, c1); ++k) {
      const int i = k - c0, t = sT[i];
      const double *D = sD + 4 * i;
      const double u = x[t], v = x[nt + t];
      b1 += c.c1L * (D[1] * u + c.sL * D[0] * v) - c.c1Y * (D[3] * u + c.sY * D[2] * v);
      b2 += sW[i] * u + c.sL * sKt[2 * i] * v - c.sY * sKt[2 * i + 1] * v;
    }
    __syncthreads();
  }
  if (!act) return;
  y[s] = c.d1 * area[s] * x[s] + a1 + b1;
  y[nt + s] = c.d2 * area[s] * x[nt + s] + c.c2 * (a2 + b2);
}

// FP64 1/sqrt(x) for x > 0: the hardware estimate refined by two
// Newton-Raphson steps y <- y (3/2 - (x/2) y^2) (each roughly doubles the
// number of correct bits of the ~23-bit estimate).
__device__ inline double rsqrt_fp64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h, y * y, 1.5);
  y = y * fma(-h, y * y, 1.5);
  return y;
}

// n . grad of the FP64 Coulomb sum at the quadrature points (the derivative
// formulation's second right-hand side): out_i = -sum_j sig_j n_i.(x_i -
// y_j)/(4 pi r^3), n_i the normal of point i's triangle.
__global__ __launch_bounds__(256) void k_direct_ngrad(int64_t nt, int nq, const double *__restrict__ tx,
                                                      const double *__restrict__ normal, int64_t ns,
                                                      const double *__restrict__ sy, const double *__restrict__ sig,
                                                      double *__restrict__ out) {
  __shared__ double sx[256], syy[256], sz[256], ss[256];
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  const bool act = i < nt;
  const double xi = act ? tx[3 * i] : 0, yi = act ? tx[3 * i + 1] : 0, zi = act ? tx[3 * i + 2] : 0;
  const int64_t tri = act ? i / nq : 0;
  const double n0 = normal[3 * tri], n1 = normal[3 * tri + 1], n2 = normal[3 * tri + 2];
  double acc = 0;
  for (int64_t j0 = 0; j0 < ns; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    if (j < ns) {
      sx[threadIdx.x] = sy[3 * j];
      syy[threadIdx.x] = sy[3 * j + 1];
      sz[threadIdx.x] = sy[3 * j + 2];
      ss[threadIdx.x] = sig[j];
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(256, ns - j0);
    for (int k = 0; k < cnt; ++k) {
      const double ax = xi - sx[k], ay = yi - syy[k], az = zi - sz[k];
      const double r2 = ax * ax + ay * ay + az * az;
      if (r2 > 0) {
        const double ir = rsqrt_fp64(r2);
        acc -= ss[k] * (n0 * ax + n1 * ay + n2 * az) * ir * ir * ir;
      }
    }
    __syncthreads();
  }
  if (act) out[i] = acc / FOUR_PI;
}

__global__ void k_rhs_assemble2(int64_t nt, int nq, const double *__restrict__ qw, const double *__restrict__ f,
                                double *__restrict__ b) {
  const int64_t s = blockIdx.x * 256ll + threadIdx.x;
  if (s >= nt) return;
  double acc = 0;
  for (int a = 0; a < nq; ++a) acc += qw[s * nq + a] * f[s * nq + a];
  b[nt + s] = acc;
}

// FP64 direct sum with monopole and dipole sources:
//   out_i = sum_j sig_j / (4 pi r) - dip_j . (x_i - y_j) / (4 pi r^3), r > 0,
// over the source chunk [blockIdx.y * chunk, (blockIdx.y + 1) * chunk) into
// out[blockIdx.y * nt + i] (a few targets and many sources run as many
// chunks, summed in chunk order by k_sum_chunks).
__global__ __launch_bounds__(256) void k_direct_md(int64_t nt, const double *__restrict__ tx, int64_t ns,
                                                   const double *__restrict__ sy, const double *__restrict__ sig,
                                                   const double *__restrict__ dip, int64_t chunk,
                                                   double *__restrict__ out) {
  __shared__ double sx[256], syy[256], sz[256], ss[256], dx[256], dyy[256], dz[256];
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  const bool act = i < nt;
  const double xi = act ? tx[3 * i] : 0, yi = act ? tx[3 * i + 1] : 0, zi = act ? tx[3 * i + 2] : 0;
  const int64_t jb = (int64_t)blockIdx.y * chunk, je = min(ns, jb + chunk);
  double acc = 0;
  for (int64_t j0 = jb; j0 < je; j0 += 256) {
    const int64_t j = j0 + threadIdx.x;
    if (j < je) {
      sx[threadIdx.x] = sy[3 * j];
      syy[threadIdx.x] = sy[3 * j + 1];
      sz[threadIdx.x] = sy[3 * j + 2];
      ss[threadIdx.x] = sig[j];
      dx[threadIdx.x] = dip ? dip[3 * j] : 0.0;
      dyy[threadIdx.x] = dip ? dip[3 * j + 1] : 0.0;
      dz[threadIdx.x] = dip ? dip[3 * j + 2] : 0.0;
    }
    __syncthreads();
    const int cnt = (int)min<int64_t>(256, je - j0);
    for (int k = 0; k < cnt; ++k) {
      const double ax = xi - sx[k], ay = yi - syy[k], az = zi - sz[k];
      const double r2 = ax * ax + ay * ay + az * az;
      if (r2 > 0) {
        const double ir = rsqrt_fp64(r2);
        acc += ss[k] * ir - (dx[k] * ax + dyy[k] * ay + dz[k] * az) * ir * ir * ir;
      }
    }
    __syncthreads();
  }
  if (act) out[(int64_t)blockIdx.y * nt + i] = acc / FOUR_PI;
}

// out[i] = sum over c < nchunk of part[c * n + i], in chunk order.
__global__ void k_sum_chunks(int64_t n, int nchunk, const double *__restrict__ part, double *__restrict__ out) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= n) return;
  double acc = 0;
  for (int c = 0; c < nchunk; ++c) acc += part[(int64_t)c * n + i];
  out[i] = acc;
}

__global__ void k_rhs_assemble(int64_t nt, int nq, const double *__restrict__ qw, const double *__restrict__ f,
                               double *__restrict__ b) {
  const int64_t s = blockIdx.x * 256ll + threadIdx.x;
  if (s >= nt) return;
  double acc = 0;
  for (int a = 0; a < nq; ++a) acc += qw[s * nq + a] * f[s * nq + a];
  b[s] = acc;
  b[nt + s] = 0.0;
}

__global__ void k_energy_sources(int64_t nt, int nq, const double *__restrict__ x, double vscale,
                                 const double *__restrict__ qw, const double *__restrict__ normal,
                                 double *__restrict__ sig, double *__restrict__ dip) {
  const int64_t i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= nt * nq) return;
  const int64_t t = i / nq;
  sig[i] = qw[i] * vscale * x[nt + t];
  const double mu = qw[i] * x[t];
  dip[3 * i] = mu * normal[3 * t];
  dip[3 * i + 1] = mu * normal[3 * t + 1];
  dip[3 * i + 2] = mu * normal[3 * t + 2];
}

// ---------------------------------------------------------------------------
// FP64 vector kernels for GMRES (fixed reduction order: deterministic)
// ---------------------------------------------------------------------------
constexpr int RED_BLOCKS = 512;

// partial[r * RED_BLOCKS + b] = sum over block b's chunk of V_r . w
__global__ __launch_bounds__(256) void k_multidot(const double *__restrict__ V, int64_t n,
                                                  const double *__restrict__ w, double *__restrict__ partial) {
  __shared__ double red[256];
  const int r = blockIdx.y;
  const int64_t chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
  const int64_t e0 = blockIdx.x * chunk, e1 = min<int64_t>(n, e0 + chunk);
  const double *v = V + (int64_t)r * n;
  double acc = 0;
  for (int64_t e = e0 + threadIdx.x; e < e1; e += 256) acc += v[e] * w[e];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(int64_t)r * RED_BLOCKS + blockIdx.x] = red[0];
}

__global__ void k_sum_partials(int nrow, const double *__restrict__ partial, double *__restrict__ out) {
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= nrow) return;
  double acc = 0;
  for (int b = 0; b < RED_BLOCKS; ++b) acc += partial[(int64_t)r * RED_BLOCKS + b];
  out[r] = acc;
}

// w -= sum_r h_r V_r
__global__ void k_sub_combo(const double *__restrict__ V, int nrow, int64_t n, const double *__restrict__ h,
                            double *__restrict__ w) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e >= n) return;
  double acc = 0;
  for (int r = 0; r < nrow; ++r) acc += h[r] * V[(int64_t)r * n + e];
  w[e] -= acc;
}

// out = sum_r y_r V_r
__global__ void k_combo(const double *__restrict__ V, int nrow, int64_t n, const double *__restrict__ y,
                        double *__restrict__ out) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e >= n) return;
  double acc = 0;
  for (int r = 0; r < nrow; ++r) acc += y[r] * V[(int64_t)r * n + e];
  out[e] = acc;
}

__global__ void k_axpby(int64_t n, double a, const double *__restrict__ x, double b, const double *__restrict__ y,
                        double *__restrict__ out) {
  const int64_t e = blockIdx.x * 256ll + threadIdx.x;
  if (e < n) out[e] = a * x[e] + b * y[e];
}

__global__ void k_energy_reduce(int64_t nq, const double *__restrict__ q, const double *__restrict__ phi,
                                double *__restrict__ out) {
  __shared__ double red[1024];
  double acc = 0;
  for (int64_t k = threadIdx.x; k < nq; k += 1024) acc += q[k] * phi[k];
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int st = 512; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = 0.5 * red[0] * FOUR_PI * KCAL;
}

inline unsigned blocks(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

}  // namespace

struct bem_op {
  int64_t nt = 0, nv = 0, N = 0, npair = 0;
  int nq = 0, precision = 0;
  double eps_in = 0, eps_out = 0, kappa = 0;
  fmm_plan *fl = nullptr, *fy = nullptr;
  double *d_tri = nullptr, *d_normal = nullptr, *d_area = nullptr, *d_qw = nullptr, *d_qpts = nullptr;
  int32_t *d_sp_off = nullptr, *d_sp_idx = nullptr;
  double *d_D = nullptr, *d_sdiag = nullptr, *d_pre = nullptr;
  // derivative formulation: W_Y - W_L corrections and diagonal, transposed pair index
  int formulation = 0, precond = 0;
  double *d_Dw = nullptr, *d_sdiag_w = nullptr;
  int32_t *d_sp_tr = nullptr;
  // P1 elements (FMM_BEM_EXTERIOR_P1): nu = nv unknowns per block (nt for
  // P0), the triangles' vertex indices, per vertex its corners (3 s + a,
  // ascending), the regular rule, and pair-minor arrays: the S - C blocks
  // (45 per pair; FP32 for single-precision operators), the K' blocks from
  // the transposed pairs (18 per pair, same type) and
  // the per-pair row terms of a matvec (6 per pair); the per-corner row sums
  bool p1 = false;
  int64_t nu = 0;
  int32_t *d_tris = nullptr, *d_vt_off = nullptr, *d_vt_list = nullptr;
  double *d_rq = nullptr, *d_P = nullptr, *d_cb = nullptr;
  void *d_B = nullptr, *d_KT = nullptr;  // FP64 for FP64 operators, FP32 otherwise
  void *q4 = nullptr, *potl = nullptr, *poty = nullptr, *gradl = nullptr, *grady = nullptr;
  // GMRES / energy scratch
  double *d_partial = nullptr, *d_h = nullptr, *d_V = nullptr, *d_z = nullptr, *d_w = nullptr, *d_r = nullptr,
         *d_xc = nullptr;
  int64_t V_rows = 0;
  std::vector<void *> allocs;
};

namespace {

int balloc(bem_op *op, void **p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes ? bytes : 16);
  if (e != hipSuccess) {
    set_error("bem: hipMalloc(" + std::to_string(bytes) + "): " + hipGetErrorString(e));
    *p = nullptr;
    return FMM_ENOMEM;
  }
  op->allocs.push_back(*p);
  return FMM_OK;
}

template <typename V>
int bupload(bem_op *op, V **p, const std::vector<V> &h) {
  int rc = balloc(op, (void **)p, h.size() * sizeof(V));
  if (rc) return rc;
  if (!h.empty()) FMM_HIP_TRY(hipMemcpy(*p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice));
  return FMM_OK;
}

int ensure_krylov(bem_op *op, int64_t rows) {
  if (op->V_rows >= rows) return FMM_OK;
  const int64_t n = 2 * op->nu;
  int rc;
  if ((rc = balloc(op, (void **)&op->d_V, (size_t)rows * n * sizeof(double)))) return rc;
  if ((rc = balloc(op, (void **)&op->d_partial, (size_t)rows * RED_BLOCKS * sizeof(double)))) return rc;
  if ((rc = balloc(op, (void **)&op->d_h, (size_t)rows * sizeof(double)))) return rc;
  op->V_rows = rows;
  return FMM_OK;
}

// dot products of the first `rows` Krylov vectors (or any rows-by-n block)
// with w; result on the host
int multidot(bem_op *op, const double *V, int rows, const double *w, double *h_host, hipStream_t s) {
  const int64_t n = 2 * op->nu;
  hipLaunchKernelGGL(k_multidot, dim3(RED_BLOCKS, rows), dim3(256), 0, s, V, n, w, op->d_partial);
  hipLaunchKernelGGL(k_sum_partials, dim3(blocks(rows, 64)), dim3(64), 0, s, rows, op->d_partial, op->d_h);
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipMemcpyAsync(h_host, op->d_h, rows * sizeof(double), hipMemcpyDeviceToHost, s));
  FMM_HIP_TRY(hipStreamSynchronize(s));
  return FMM_OK;
}

// (Re)build the per-triangle 2 x 2 preconditioner blocks of kind `kind`.
int precond_setup(bem_op *op, int kind, hipStream_t s) {
  const int64_t nt = op->nt;
  if (op->p1) {
    if (kind != FMM_BEM_PRECOND_MASS) {
      set_error("bem: P1 elements take the (lumped) mass preconditioner only");
      return FMM_EINVAL;
    }
    hipLaunchKernelGGL(k_precond_setup_lumped, dim3(blocks(op->nv)), dim3(256), 0, s, op->nv, op->d_vt_off,
                       op->d_vt_list, op->d_area, op->d_pre);
  } else if (kind == FMM_BEM_PRECOND_MASS)
    hipLaunchKernelGGL(k_precond_setup_mass, dim3(blocks(nt)), dim3(256), 0, s, nt, op->d_area, op->d_pre);
  else if (op->formulation != FMM_BEM_DIRECT)
    hipLaunchKernelGGL(k_precond_setup_deriv, dim3(blocks(nt)), dim3(256), 0, s, nt, op->d_area, op->d_sdiag,
                       op->d_sdiag_w, deriv_coef(op->formulation, op->eps_in, op->eps_out), op->d_pre);
  else
    hipLaunchKernelGGL(k_precond_setup, dim3(blocks(nt)), dim3(256), 0, s, nt, op->d_area, op->d_sdiag,
                       op->eps_in / op->eps_out, op->d_pre);
  FMM_HIP_TRY(hipGetLastError());
  op->precond = kind;
  return FMM_OK;
}

}  // namespace

extern "C" {

int bem_setup(const double *verts, int64_t nv, const int32_t *tris, int64_t nt, int quad_pts, double eps_in,
              double eps_out, double kappa, int p, int ncrit, int precision, int formulation, fmm_stream_t stream,
              bem_op **out) {
  if (!out) { set_error("bem_setup: out is NULL"); return FMM_EINVAL; }
  *out = nullptr;
  if (formulation != FMM_BEM_DIRECT && formulation != FMM_BEM_DERIVATIVE && formulation != FMM_BEM_EXTERIOR &&
      formulation != FMM_BEM_EXTERIOR_P1) {
    set_error("bem_setup: unknown formulation");
    return FMM_EINVAL;
  }
  if (nv <= 0 || nt <= 0 || !verts || !tris) { set_error("bem_setup: empty or null mesh"); return FMM_EINVAL; }
  if (quad_pts != 3 && quad_pts != 6) { set_error("bem_setup: quad_pts must be 3 or 6"); return FMM_EINVAL; }
  if (!(eps_in > 0) || !(eps_out > 0) || !std::isfinite(eps_in) || !std::isfinite(eps_out)) {
    set_error("bem_setup: permittivities must be positive");
    return FMM_EINVAL;
  }
  if (!(kappa >= 0) || !std::isfinite(kappa)) { set_error("bem_setup: kappa must be finite and >= 0"); return FMM_EINVAL; }
  if (nt * quad_pts > 0x7fffffffll) { set_error("bem_setup: too many quadrature points"); return FMM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  bem_op *op = new (std::nothrow) bem_op();
  if (!op) { set_error("bem_setup: out of host memory"); return FMM_ENOMEM; }
  op->nt = nt; op->nv = nv; op->nq = quad_pts; op->N = nt * quad_pts; op->precision = precision;
  op->eps_in = eps_in; op->eps_out = eps_out; op->kappa = kappa;
  op->formulation = formulation;
  op->p1 = formulation == FMM_BEM_EXTERIOR_P1;
  op->nu = op->p1 ? nv : nt;
  const bool deriv = formulation != FMM_BEM_DIRECT;
  int rc = FMM_OK;
  do {
    // geometry on the host
    std::vector<double> tri(nt * 9), normal(nt * 3), area(nt), qw(op->N), qpts(op->N * 3);
    std::vector<double> rq;
    regular(quad_pts, rq);
    bool bad = false;
    for (int64_t t = 0; t < nt; ++t) {
      double v[3][3];
      for (int i = 0; i < 3; ++i) {
        const int32_t vi = tris[3 * t + i];
        if (vi < 0 || vi >= nv) { bad = true; break; }
        for (int d = 0; d < 3; ++d) { v[i][d] = verts[3 * vi + d]; tri[t * 9 + 3 * i + d] = v[i][d]; }
      }
      if (bad) break;
      const double e1[3] = {v[1][0] - v[0][0], v[1][1] - v[0][1], v[1][2] - v[0][2]};
      const double e2[3] = {v[2][0] - v[0][0], v[2][1] - v[0][1], v[2][2] - v[0][2]};
      const double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
      const double cn = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      if (!(cn > 0) || !std::isfinite(cn)) { bad = true; break; }
      area[t] = 0.5 * cn;
      for (int d = 0; d < 3; ++d) normal[3 * t + d] = c[d] / cn;
      for (int a = 0; a < quad_pts; ++a) {
        const double l1 = rq[3 * a], l2 = rq[3 * a + 1], w = rq[3 * a + 2];
        for (int d = 0; d < 3; ++d) qpts[(t * quad_pts + a) * 3 + d] = (1 - l1 - l2) * v[0][d] + l1 * v[1][d] + l2 * v[2][d];
        qw[t * quad_pts + a] = w * area[t];
      }
    }
    if (bad) { set_error("bem_setup: bad vertex index or degenerate triangle"); rc = FMM_EINVAL; break; }
    // pairs of triangles that share a vertex (identical included), s-major
    std::vector<std::vector<int32_t>> vt(nv);
    for (int64_t t = 0; t < nt; ++t)
      for (int i = 0; i < 3; ++i) vt[tris[3 * t + i]].push_back((int32_t)t);
    std::vector<int32_t> off(nt + 1, 0), idx, ps;
    std::vector<int32_t> nb;
    for (int64_t t = 0; t < nt; ++t) {
      nb.clear();
      for (int i = 0; i < 3; ++i) nb.insert(nb.end(), vt[tris[3 * t + i]].begin(), vt[tris[3 * t + i]].end());
      std::sort(nb.begin(), nb.end());
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      idx.insert(idx.end(), nb.begin(), nb.end());
      ps.insert(ps.end(), nb.size(), (int32_t)t);
      off[t + 1] = (int32_t)idx.size();
    }
    op->npair = (int64_t)idx.size();
    // index of the transposed pair (t, s) of every pair (s, t)
    std::vector<int32_t> tr(idx.size());
    for (int64_t t = 0; t < nt; ++t)
      for (int32_t k = off[t]; k < off[t + 1]; ++k) {
        const int32_t u = idx[k];
        tr[k] = (int32_t)(std::lower_bound(idx.begin() + off[u], idx.begin() + off[u + 1], (int32_t)t) - idx.begin());
      }
    if ((rc = bupload(op, &op->d_tri, tri))) break;
    if ((rc = bupload(op, &op->d_normal, normal))) break;
    if ((rc = bupload(op, &op->d_area, area))) break;
    if ((rc = bupload(op, &op->d_qw, qw))) break;
    if ((rc = bupload(op, &op->d_qpts, qpts))) break;
    if ((rc = bupload(op, &op->d_sp_off, off))) break;
    if ((rc = bupload(op, &op->d_sp_idx, idx))) break;
    int32_t *d_ps = nullptr;
    if ((rc = bupload(op, &d_ps, ps))) break;
    std::vector<double> ro, rr;
    collapsed(NO, ro);
    collapsed(NREM, rr);
    double *d_ro = nullptr, *d_rr = nullptr, *d_rq = nullptr;
    if ((rc = bupload(op, &d_ro, ro))) break;
    if ((rc = bupload(op, &d_rr, rr))) break;
    if ((rc = bupload(op, &d_rq, rq))) break;
    op->d_rq = d_rq;
    if ((rc = balloc(op, (void **)&op->d_pre, op->nu * 4 * sizeof(double)))) break;
    if (deriv && (rc = bupload(op, &op->d_sp_tr, tr))) break;
    if (op->p1) {
      // per vertex its triangle corners 3 s + a, ascending; every vertex
      // must belong to a triangle (it carries two unknowns)
      std::vector<int32_t> tv(tris, tris + 3 * nt), voff(nv + 1, 0), vlist(3 * nt);
      for (int64_t c = 0; c < 3 * nt; ++c) ++voff[tv[c] + 1];
      bool lone = false;
      for (int64_t i = 0; i < nv; ++i) {
        lone = lone || voff[i + 1] == 0;
        voff[i + 1] += voff[i];
      }
      if (lone) { set_error("bem_setup: P1 elements need every vertex on a triangle"); rc = FMM_EINVAL; break; }
      std::vector<int32_t> fill(voff.begin(), voff.end() - 1);
      for (int64_t c = 0; c < 3 * nt; ++c) vlist[fill[tv[c]]++] = (int32_t)c;
      if ((rc = bupload(op, &op->d_tris, tv))) break;
      if ((rc = bupload(op, &op->d_vt_off, voff))) break;
      if ((rc = bupload(op, &op->d_vt_list, vlist))) break;
      const size_t bs = precision == FMM_FP64 ? sizeof(double) : sizeof(float);
      if ((rc = balloc(op, &op->d_B, op->npair * 45 * bs))) break;
      if ((rc = balloc(op, &op->d_KT, op->npair * 18 * bs))) break;
      if ((rc = balloc(op, (void **)&op->d_P, op->npair * 6 * sizeof(double)))) break;
      if ((rc = balloc(op, (void **)&op->d_cb, nt * 6 * sizeof(double)))) break;
      if (precision == FMM_FP64) {
        hipLaunchKernelGGL(k_singular_p1<double>, dim3(blocks(op->npair, 128)), dim3(128), 0, s, op->npair, d_ps,
                           op->d_sp_idx, op->d_tri, op->d_normal, op->d_area, d_ro, NO * NO, d_rr, NREM * NREM,
                           d_rq, quad_pts, kappa, (double *)op->d_B);
        hipLaunchKernelGGL(k_p1_transpose<double>, dim3(blocks(op->npair)), dim3(256), 0, s, op->npair,
                           op->d_sp_tr, (const double *)op->d_B, (double *)op->d_KT);
      } else {
        hipLaunchKernelGGL(k_singular_p1<float>, dim3(blocks(op->npair, 128)), dim3(128), 0, s, op->npair, d_ps,
                           op->d_sp_idx, op->d_tri, op->d_normal, op->d_area, d_ro, NO * NO, d_rr, NREM * NREM,
                           d_rq, quad_pts, kappa, (float *)op->d_B);
        hipLaunchKernelGGL(k_p1_transpose<float>, dim3(blocks(op->npair)), dim3(256), 0, s, op->npair,
                           op->d_sp_tr, (const float *)op->d_B, (float *)op->d_KT);
      }
    } else {
      if ((rc = balloc(op, (void **)&op->d_D, op->npair * 4 * sizeof(double)))) break;
      if ((rc = balloc(op, (void **)&op->d_sdiag, nt * 2 * sizeof(double)))) break;
      if (deriv) {
        if ((rc = balloc(op, (void **)&op->d_Dw, op->npair * sizeof(double)))) break;
        if ((rc = balloc(op, (void **)&op->d_sdiag_w, nt * sizeof(double)))) break;
      }
      hipLaunchKernelGGL(k_singular, dim3(blocks(op->npair, 128)), dim3(128), 0, s, op->npair, d_ps, op->d_sp_idx,
                         op->d_tri, op->d_normal, op->d_area, d_ro, NO * NO, d_rr, NREM * NREM, d_rq, quad_pts,
                         kappa, op->d_D, op->d_sdiag, deriv ? 1 : 0, op->d_Dw, op->d_sdiag_w);
    }
    if (hipGetLastError() != hipSuccess) { set_error("bem_setup: launch failed"); rc = FMM_EHIP; break; }
    if ((rc = precond_setup(op, op->p1 ? FMM_BEM_PRECOND_MASS : FMM_BEM_PRECOND_BLOCK, s))) break;
    // the two FMM plans on the quadrature points
    if ((rc = fmm_setup(op->d_qpts, op->N, FMM_LAPLACE, 0.0, p, ncrit, precision, stream, &op->fl))) break;
    if ((rc = fmm_setup(op->d_qpts, op->N, FMM_YUKAWA, kappa, p, ncrit, precision, stream, &op->fy))) break;
    const size_t es = precision == FMM_FP64 ? 8 : 4;
    // charges (N) and dipoles (3N); one potential per point and kernel
    if ((rc = balloc(op, &op->q4, 4 * op->N * es))) break;
    if ((rc = balloc(op, &op->potl, op->N * es))) break;
    if ((rc = balloc(op, &op->poty, op->N * es))) break;
    if (deriv) {
      if ((rc = balloc(op, &op->gradl, 3 * op->N * es))) break;
      if ((rc = balloc(op, &op->grady, 3 * op->N * es))) break;
    }
    if ((rc = balloc(op, (void **)&op->d_z, 2 * op->nu * sizeof(double)))) break;
    if ((rc = balloc(op, (void **)&op->d_w, 2 * op->nu * sizeof(double)))) break;
    if ((rc = balloc(op, (void **)&op->d_r, 2 * op->nu * sizeof(double)))) break;
    if ((rc = balloc(op, (void **)&op->d_xc, 2 * op->nu * sizeof(double)))) break;
    if ((rc = ensure_krylov(op, 2))) break;
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess) { set_error(std::string("bem_setup: ") + hipGetErrorString(e)); rc = FMM_EHIP; }
  } while (0);
  if (rc) { bem_free(op); return rc; }
  *out = op;
  return FMM_OK;
}

int bem_matvec(bem_op *op, const double *x, double *y, fmm_stream_t stream) {
  if (!op || !x || !y) { set_error("bem_matvec: null argument"); return FMM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = op->N, nt = op->nt;
  int rc;
  const double er = op->eps_in / op->eps_out;
  const DerivCoef dc = deriv_coef(op->formulation, op->eps_in, op->eps_out);
  const bool deriv = op->formulation != FMM_BEM_DIRECT;
  // one pass per kernel: single layer as charges, double layer as dipoles
  // (the four-column form would need potentials and gradients of four)
  const int64_t Nq = (int64_t)nt * op->nq;
  if (op->p1) {
    const size_t es = op->precision == FMM_FP64 ? 8 : 4;
    const char *qq = (const char *)op->q4;
    if (op->precision == FMM_FP64)
      hipLaunchKernelGGL(k_p1_src<double>, dim3(blocks(N)), dim3(256), 0, s, nt, op->nq, op->d_tris, op->d_rq, x,
                         op->nv, 1.0, op->d_qw, op->d_normal, (double *)op->q4, (double *)op->q4 + Nq);
    else
      hipLaunchKernelGGL(k_p1_src<float>, dim3(blocks(N)), dim3(256), 0, s, nt, op->nq, op->d_tris, op->d_rq, x,
                         op->nv, 1.0, op->d_qw, op->d_normal, (float *)op->q4, (float *)op->q4 + Nq);
    FMM_HIP_TRY(hipGetLastError());
    if ((rc = fmm_eval_pair_md(op->fl, op->fy, qq, qq + Nq * es, dc.sL, dc.sY, op->potl, op->gradl, op->poty,
                               op->grady, s)))
      return rc;
    if (op->precision == FMM_FP64)
      hipLaunchKernelGGL(k_p1_pairs<double>, dim3(blocks(op->npair)), dim3(256), 0, s, op->npair, op->d_sp_idx,
                         op->d_tris, (const double *)op->d_B, (const double *)op->d_KT, x, op->nv, dc, op->d_P);
    else
      hipLaunchKernelGGL(k_p1_pairs<float>, dim3(blocks(op->npair)), dim3(256), 0, s, op->npair, op->d_sp_idx,
                         op->d_tris, (const float *)op->d_B, (const float *)op->d_KT, x, op->nv, dc, op->d_P);
    if (op->precision == FMM_FP64)
      hipLaunchKernelGGL(k_p1_corner<double>, dim3(blocks(nt, 64)), dim3(64), 0, s, nt, op->nq, (const double *)op->potl,
                         (const double *)op->gradl, (const double *)op->poty, (const double *)op->grady, op->d_qw,
                         op->d_rq, op->d_area, op->d_normal, op->d_tris, op->d_sp_off, op->npair, op->d_P, x, op->nv,
                         dc, op->d_cb);
    else
      hipLaunchKernelGGL(k_p1_corner<float>, dim3(blocks(nt, 64)), dim3(64), 0, s, nt, op->nq, (const float *)op->potl,
                         (const float *)op->gradl, (const float *)op->poty, (const float *)op->grady, op->d_qw,
                         op->d_rq, op->d_area, op->d_normal, op->d_tris, op->d_sp_off, op->npair, op->d_P, x, op->nv,
                         dc, op->d_cb);
    hipLaunchKernelGGL(k_p1_gather, dim3(blocks(op->nv)), dim3(256), 0, s, op->nv, op->d_vt_off, op->d_vt_list,
                       op->d_cb, y);
    FMM_HIP_TRY(hipGetLastError());
    return FMM_OK;
  }
  if (op->precision == FMM_FP64) {
    double *qq = (double *)op->q4;
    hipLaunchKernelGGL(k_bem_p1_md<double>, dim3(blocks(N)), dim3(256), 0, s, nt, op->nq, x, op->d_qw, op->d_normal,
                       qq, qq + Nq);
  } else {
    float *qq = (float *)op->q4;
    hipLaunchKernelGGL(k_bem_p1_md<float>, dim3(blocks(N)), dim3(256), 0, s, nt, op->nq, x, op->d_qw, op->d_normal,
                       qq, qq + Nq);
  }
  FMM_HIP_TRY(hipGetLastError());
  {
    const size_t es = op->precision == FMM_FP64 ? 8 : 4;
    const char *qq = (const char *)op->q4;
    if ((rc = fmm_eval_pair_md(op->fl, op->fy, qq, qq + Nq * es, deriv ? dc.sL : -1.0, deriv ? dc.sY : -er,
                               op->potl, op->gradl, op->poty, op->grady, s)))
      return rc;
  }
  if (deriv) {
    if (op->precision == FMM_FP64)
      hipLaunchKernelGGL(k_bem_p2_deriv<double>, dim3(blocks(nt, 64)), dim3(64), 0, s, nt, op->nq,
                         (const double *)op->potl, (const double *)op->gradl, (const double *)op->poty,
                         (const double *)op->grady, op->d_qw, op->d_area, op->d_normal, op->d_sp_off, op->d_sp_idx,
                         op->d_sp_tr, op->d_D, op->d_Dw, x, dc, y);
    else
      hipLaunchKernelGGL(k_bem_p2_deriv<float>, dim3(blocks(nt, 64)), dim3(64), 0, s, nt, op->nq,
                         (const float *)op->potl, (const float *)op->gradl, (const float *)op->poty,
                         (const float *)op->grady, op->d_qw, op->d_area, op->d_normal, op->d_sp_off, op->d_sp_idx,
                         op->d_sp_tr, op->d_D, op->d_Dw, x, dc, y);
    FMM_HIP_TRY(hipGetLastError());
    return FMM_OK;
  }
  if (op->precision == FMM_FP64) {
    hipLaunchKernelGGL(k_bem_p2_md<double>, dim3(blocks(nt, 64)), dim3(64), 0, s, nt, op->nq, (const double *)op->potl,
                       (const double *)op->poty, op->d_qw, op->d_area, op->d_sp_off, op->d_sp_idx, op->d_D, x, er, y);
  } else {
    hipLaunchKernelGGL(k_bem_p2_md<float>, dim3(blocks(nt, 64)), dim3(64), 0, s, nt, op->nq, (const float *)op->potl,
                       (const float *)op->poty, op->d_qw, op->d_area, op->d_sp_off, op->d_sp_idx, op->d_D, x, er, y);
  }
  FMM_HIP_TRY(hipGetLastError());
  return FMM_OK;
}

int bem_set_preconditioner(bem_op *op, int kind, fmm_stream_t stream) {
  if (!op) { set_error("bem_set_preconditioner: null operator"); return FMM_EINVAL; }
  if (kind != FMM_BEM_PRECOND_BLOCK && kind != FMM_BEM_PRECOND_MASS) {
    set_error("bem_set_preconditioner: unknown preconditioner");
    return FMM_EINVAL;
  }
  return precond_setup(op, kind, (hipStream_t)stream);
}

int bem_precondition(bem_op *op, const double *x, double *y, fmm_stream_t stream) {
  if (!op || !x || !y) { set_error("bem_precondition: null argument"); return FMM_EINVAL; }
  hipLaunchKernelGGL(k_precond_apply, dim3(blocks(op->nu)), dim3(256), 0, (hipStream_t)stream, op->nu, op->d_pre, x, y);
  FMM_HIP_TRY(hipGetLastError());
  return FMM_OK;
}

// The right-hand side's launches; sig (nq) and f (the operator's N
// quadrature points) are temporary arrays that every launch writes before
// it is read.
static int rhs_core(bem_op *op, const double *qxyz, const double *q, int64_t nq, double *b, double *sig, double *f,
                    hipStream_t s) {
  // sigma_k = q_k / eps_in (q_k / eps_out for the exterior formulation)
  const double eps = op->formulation == FMM_BEM_EXTERIOR || op->p1 ? op->eps_out : op->eps_in;
  hipLaunchKernelGGL(k_axpby, dim3(blocks(std::max<int64_t>(1, nq))), dim3(256), 0, s, nq, 1.0 / eps, q, 0.0, q, sig);
  hipLaunchKernelGGL(k_direct_md, dim3(blocks(op->N), 1), dim3(256), 0, s, op->N, op->d_qpts, nq, qxyz, sig,
                     (const double *)nullptr, std::max<int64_t>(1, nq), f);
  if (op->p1) {
    // both fields tested with the hat functions, then added into the vertices
    hipLaunchKernelGGL(k_p1_project, dim3(blocks(op->nt)), dim3(256), 0, s, op->nt, op->nq, op->d_qw, op->d_rq, f, 0,
                       op->d_cb);
    hipLaunchKernelGGL(k_direct_ngrad, dim3(blocks(op->N)), dim3(256), 0, s, op->N, op->nq, op->d_qpts, op->d_normal,
                       nq, qxyz, sig, f);
    hipLaunchKernelGGL(k_p1_project, dim3(blocks(op->nt)), dim3(256), 0, s, op->nt, op->nq, op->d_qw, op->d_rq, f, 1,
                       op->d_cb);
    hipLaunchKernelGGL(k_p1_gather, dim3(blocks(op->nv)), dim3(256), 0, s, op->nv, op->d_vt_off, op->d_vt_list,
                       op->d_cb, b);
  } else {
    hipLaunchKernelGGL(k_rhs_assemble, dim3(blocks(op->nt)), dim3(256), 0, s, op->nt, op->nq, op->d_qw, f, b);
  }
  if (op->formulation != FMM_BEM_DIRECT && !op->p1) {
    // second block: the normal derivative of the same Coulomb sum
    hipLaunchKernelGGL(k_direct_ngrad, dim3(blocks(op->N)), dim3(256), 0, s, op->N, op->nq, op->d_qpts, op->d_normal,
                       nq, qxyz, sig, f);
    hipLaunchKernelGGL(k_rhs_assemble2, dim3(blocks(op->nt)), dim3(256), 0, s, op->nt, op->nq, op->d_qw, f, b);
  }
  FMM_HIP_TRY(hipGetLastError());
  return FMM_OK;
}

int bem_rhs(bem_op *op, const double *qxyz, const double *q, int64_t nq, double *b, fmm_stream_t stream) {
  if (!op || !b || nq < 0 || (nq > 0 && (!qxyz || !q))) { set_error("bem_rhs: bad argument"); return FMM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  double *sig = nullptr, *f = nullptr;
  FMM_HIP_TRY(hipMallocAsync((void **)&sig, std::max<int64_t>(1, nq) * sizeof(double), s));
  FMM_HIP_TRY(hipMallocAsync((void **)&f, op->N * sizeof(double), s));
  const int rc = rhs_core(op, qxyz, q, nq, b, sig, f, s);
  (void)hipFreeAsync(sig, s);
  (void)hipFreeAsync(f, s);
  return rc;
}

// Scratch of bem_rhs_noalloc: its two temporary arrays (scaled charges, then
// the field at the quadrature points, 256-byte aligned) in one static device
// array per GPU, held until the process ends.  Host code never passes the
// array's name (a host-side stand-in) to a launch: the device address comes
// from hipGetSymbolAddress, once per device, with that device current.
static __device__ __align__(256) double scratch[BEM_RHS_SCRATCH_DOUBLES];

static std::mutex g_scratch_mu;
static std::vector<double *> g_scratch_dev;  // per device ordinal

static int scratch_address(double **out) {
  int dev = 0;
  FMM_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((int)g_scratch_dev.size() <= dev) g_scratch_dev.resize(dev + 1, nullptr);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error(std::string("bem_rhs_noalloc: hipGetSymbolAddress: ") + hipGetErrorString(e));
      return FMM_EHIP;
    }
    g_scratch_dev[dev] = (double *)p;
  }
  *out = g_scratch_dev[dev];
  return FMM_OK;
}

int bem_rhs_noalloc(bem_op *op, const double *qxyz, const double *q, int64_t nq, double *b, fmm_stream_t stream) {
  if (!op || !b || nq < 0 || (nq > 0 && (!qxyz || !q))) {
    set_error("bem_rhs_noalloc: bad argument");
    return FMM_EINVAL;
  }
  const int64_t nsig = (std::max<int64_t>(1, nq) + 31) / 32 * 32;  // f starts 256-byte aligned
  if (nq > BEM_RHS_SCRATCH_DOUBLES || nsig + op->N > BEM_RHS_SCRATCH_DOUBLES) {
    set_error("bem_rhs_noalloc: " + std::to_string(nq) + " charges and " + std::to_string(op->N) +
              " quadrature points need " + std::to_string(nsig + op->N) + " doubles of scratch, more than the " +
              std::to_string(BEM_RHS_SCRATCH_DOUBLES) + " it holds");
    return FMM_EINVAL;
  }
  double *base = nullptr;
  int rc;
  if ((rc = scratch_address(&base))) return rc;
  return rhs_core(op, qxyz, q, nq, b, base, base + nsig, (hipStream_t)stream);
}

int bem_energy(bem_op *op, const double *x, const double *qxyz, const double *q, int64_t nq, double *dG,
               fmm_stream_t stream) {
  if (!op || !x || !dG || nq < 0 || (nq > 0 && (!qxyz || !q))) { set_error("bem_energy: bad argument"); return FMM_EINVAL; }
  hipStream_t s = (hipStream_t)stream;
  *dG = 0;
  if (nq == 0) return FMM_OK;
  double *sig = nullptr, *dip = nullptr, *phi = nullptr, *res = nullptr;
  FMM_HIP_TRY(hipMallocAsync((void **)&sig, op->N * sizeof(double), s));
  FMM_HIP_TRY(hipMallocAsync((void **)&dip, op->N * 3 * sizeof(double), s));
  FMM_HIP_TRY(hipMallocAsync((void **)&phi, nq * sizeof(double), s));
  FMM_HIP_TRY(hipMallocAsync((void **)&res, sizeof(double), s));
  // the exterior unknowns map to (phi_1, d phi_1/dn) by the interface
  // conditions: phi_1 = phi_2, eps_in d phi_1/dn = eps_out d phi_2/dn
  const double vscale = op->formulation == FMM_BEM_EXTERIOR || op->p1 ? op->eps_out / op->eps_in : 1.0;
  if (op->p1)
    hipLaunchKernelGGL(k_p1_src<double>, dim3(blocks(op->N)), dim3(256), 0, s, op->nt, op->nq, op->d_tris, op->d_rq,
                       x, op->nv, vscale, op->d_qw, op->d_normal, sig, dip);
  else
    hipLaunchKernelGGL(k_energy_sources, dim3(blocks(op->N)), dim3(256), 0, s, op->nt, op->nq, x, vscale, op->d_qw,
                       op->d_normal, sig, dip);
  // few targets, many sources: the sources in chunks (at least ~2,048
  // workgroups in all), partial sums added in chunk order
  const int64_t tb = blocks(nq);
  const int nchunk = (int)std::max<int64_t>(1, std::min<int64_t>((op->N + 4095) / 4096, (2048 + tb - 1) / tb));
  const int64_t chunk = (op->N + nchunk - 1) / nchunk;
  double *part = phi;
  if (nchunk > 1) FMM_HIP_TRY(hipMallocAsync((void **)&part, (size_t)nchunk * nq * sizeof(double), s));
  hipLaunchKernelGGL(k_direct_md, dim3(tb, nchunk), dim3(256), 0, s, nq, qxyz, op->N, op->d_qpts, sig, dip, chunk,
                     part);
  if (nchunk > 1) hipLaunchKernelGGL(k_sum_chunks, dim3(tb), dim3(256), 0, s, nq, nchunk, part, phi);
  hipLaunchKernelGGL(k_energy_reduce, dim3(1), dim3(1024), 0, s, nq, q, phi, res);
  FMM_HIP_TRY(hipGetLastError());
  FMM_HIP_TRY(hipMemcpyAsync(dG, res, sizeof(double), hipMemcpyDeviceToHost, s));
  FMM_HIP_TRY(hipStreamSynchronize(s));
  (void)hipFreeAsync(sig, s);
  (void)hipFreeAsync(dip, s);
  if (part != phi) (void)hipFreeAsync(part, s);
  (void)hipFreeAsync(phi, s);
  (void)hipFreeAsync(res, s);
  return FMM_OK;
}

// One GMRES run on op (right preconditioning) from x: stops at relative
// residual tol (relative to bnorm) measured with the recomputed residual.
static int gmres_core(bem_op *op, const double *b, double *x, double bnorm, double tol, int maxiter, int restart,
                      int *it_total, double *hist, int hist_cap, hipStream_t s) {
  const int64_t n = 2 * op->nu;
  int rc;
  if (restart <= 0 || restart > maxiter) restart = maxiter;
  if ((rc = ensure_krylov(op, restart + 1))) return rc;
  std::vector<double> H((size_t)(restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), h(restart + 1),
      h2(restart + 1), y(restart);
  double *V = op->d_V;
  while (true) {
    // r = b - A x
    if ((rc = bem_matvec(op, x, op->d_w, s))) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 1.0, b, -1.0, op->d_w, op->d_r);
    double rr;
    if ((rc = multidot(op, op->d_r, 1, op->d_r, &rr, s))) return rc;
    double beta = std::sqrt(rr);
    if (!std::isfinite(beta)) { set_error("gmres: non-finite residual"); return FMM_EBREAKDOWN; }
    if (beta <= tol * bnorm) return FMM_OK;
    if (*it_total >= maxiter) return FMM_ENOTCONV;
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 1.0 / beta, op->d_r, 0.0, op->d_r, V);
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int j = 0;
    for (; j < restart && *it_total < maxiter; ++j) {
      double *vj = V + (int64_t)j * n, *vn = V + (int64_t)(j + 1) * n;
      if ((rc = bem_precondition(op, vj, op->d_z, s))) return rc;
      if ((rc = bem_matvec(op, op->d_z, vn, s))) return rc;
      // classical Gram-Schmidt, twice
      if ((rc = multidot(op, V, j + 1, vn, h.data(), s))) return rc;
      FMM_HIP_TRY(hipMemcpyAsync(op->d_h, h.data(), (j + 1) * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_sub_combo, dim3(blocks(n)), dim3(256), 0, s, V, j + 1, n, op->d_h, vn);
      if ((rc = multidot(op, V, j + 1, vn, h2.data(), s))) return rc;
      FMM_HIP_TRY(hipMemcpyAsync(op->d_h, h2.data(), (j + 1) * sizeof(double), hipMemcpyHostToDevice, s));
      hipLaunchKernelGGL(k_sub_combo, dim3(blocks(n)), dim3(256), 0, s, V, j + 1, n, op->d_h, vn);
      for (int i = 0; i <= j; ++i) h[i] += h2[i];
      double ww;
      if ((rc = multidot(op, vn, 1, vn, &ww, s))) return rc;
      const double hn = std::sqrt(ww);
      if (!std::isfinite(hn)) { set_error("gmres: non-finite Arnoldi vector"); return FMM_EBREAKDOWN; }
      if (hn > 0)
        hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 1.0 / hn, vn, 0.0, vn, vn);
      // Givens rotations on the Hessenberg column
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * h[i] + sn[i] * h[i + 1];
        h[i + 1] = -sn[i] * h[i] + cs[i] * h[i + 1];
        h[i] = t;
      }
      const double den = std::hypot(h[j], hn);
      cs[j] = den > 0 ? h[j] / den : 1.0;
      sn[j] = den > 0 ? hn / den : 0.0;
      h[j] = den;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[(size_t)i * restart + j] = h[i];
      const double est = std::fabs(g[j + 1]) / bnorm;
      if (hist && *it_total < hist_cap) hist[*it_total] = est;
      ++*it_total;
      if (est <= tol || hn == 0) { ++j; break; }
    }
    // solve the triangular system and update x += P^-1 V y
    for (int i = j - 1; i >= 0; --i) {
      double t = g[i];
      for (int k = i + 1; k < j; ++k) t -= H[(size_t)i * restart + k] * y[k];
      y[i] = t / H[(size_t)i * restart + i];
    }
    FMM_HIP_TRY(hipMemcpyAsync(op->d_h, y.data(), j * sizeof(double), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_combo, dim3(blocks(n)), dim3(256), 0, s, V, j, n, op->d_h, op->d_w);
    if ((rc = bem_precondition(op, op->d_w, op->d_z, s))) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 1.0, x, 1.0, op->d_z, x);
    FMM_HIP_TRY(hipGetLastError());
  }
}

int gmres_solve(bem_op *op, bem_op *refine, const double *b, double *x, double tol, double inner_tol, int maxiter,
                int restart, int *iters, double *hist, fmm_stream_t stream) {
  if (!op || !b || !x || !(tol > 0) || maxiter < 1) { set_error("gmres_solve: bad argument"); return FMM_EINVAL; }
  if (refine == op) {
    // the refinement loop keeps its residual in the refine operator's
    // buffers, which the inner solve on `op` would overwrite
    set_error("gmres_solve: the refine operator must differ from op");
    return FMM_EINVAL;
  }
  if (refine && (refine->nt != op->nt || refine->nu != op->nu || refine->formulation != op->formulation ||
                 refine->nq != op->nq || refine->eps_in != op->eps_in || refine->eps_out != op->eps_out ||
                 refine->kappa != op->kappa)) {
    set_error("gmres_solve: refine operator on another mesh, element type, formulation, quadrature rule, "
              "permittivities or kappa");
    return FMM_EINVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int64_t n = 2 * op->nu;
  int it = 0, rc;
  double bb;
  if ((rc = multidot(op, b, 1, b, &bb, s))) return rc;
  const double bnorm = std::sqrt(bb);
  if (iters) *iters = 0;
  if (bnorm == 0) {
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 0.0, b, 0.0, b, x);
    FMM_HIP_TRY(hipStreamSynchronize(s));
    return FMM_OK;
  }
  if (!refine) {
    rc = gmres_core(op, b, x, bnorm, tol, maxiter, restart, &it, hist, maxiter, s);
    if (iters) *iters = it;
    return rc;
  }
  // iterative refinement: residuals with `refine`, corrections with `op`
  if (!(inner_tol > 0)) inner_tol = 1e-4;
  for (int outer = 0; outer < 50; ++outer) {
    if ((rc = bem_matvec(refine, x, refine->d_w, s))) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 1.0, b, -1.0, refine->d_w, refine->d_r);
    double rr;
    if ((rc = multidot(op, refine->d_r, 1, refine->d_r, &rr, s))) return rc;
    const double rn = std::sqrt(rr);
    if (!std::isfinite(rn)) { set_error("gmres: non-finite residual"); return FMM_EBREAKDOWN; }
    if (rn <= tol * bnorm) { if (iters) *iters = it; return FMM_OK; }
    if (it >= maxiter) break;
    // correction d: op d = r, from d = 0
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 0.0, b, 0.0, b, refine->d_xc);
    rc = gmres_core(op, refine->d_r, refine->d_xc, rn, inner_tol, maxiter, restart, &it, hist, maxiter, s);
    if (rc != FMM_OK && rc != FMM_ENOTCONV) return rc;
    hipLaunchKernelGGL(k_axpby, dim3(blocks(n)), dim3(256), 0, s, n, 1.0, x, 1.0, refine->d_xc, x);
    FMM_HIP_TRY(hipGetLastError());
  }
  if (iters) *iters = it;
  return FMM_ENOTCONV;
}

int bem_info(const bem_op *op, bem_info_t *o) {
  if (!op || !o) { set_error("bem_info: null argument"); return FMM_EINVAL; }
  o->n_triangles = op->nt;
  o->n_points = op->N;
  o->n_singular_pairs = op->npair;
  o->quad_pts = op->nq;
  o->precision = op->precision;
  o->formulation = op->formulation;
  o->preconditioner = op->precond;
  o->n_unknowns = op->nu;
  return FMM_OK;
}

fmm_plan *bem_fmm_plan(bem_op *op, int kernel) {
  if (!op) return nullptr;
  return kernel == FMM_YUKAWA ? op->fy : op->fl;
}

void bem_free(bem_op *op) {
  if (!op) return;
  fmm_free(op->fl);
  fmm_free(op->fy);
  for (void *p : op->allocs) (void)hipFree(p);
  delete op;
}

}  // extern "C"
