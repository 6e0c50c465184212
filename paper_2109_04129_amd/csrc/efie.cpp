// EFIE Galerkin entries with RWG basis (host).  Eqs. (2)-(3), (9) with the
// e^{jwt} convention:
//   Z_mn = jw mu <f_m, f_n G> - (j / (w eps)) <div f_m, div' f_n G>,
//   G = exp(-jkR) / (4 pi R).
// Each entry is the sum over the four triangle pairs of
//   s_P s_Q l_m l_n / (A_P A_Q) * [ (jw mu / 4) II (r - v_P).(r' - v_Q) G
//                                    - (j / (w eps)) II G ],
// evaluated only for m <= n (Z_nm := Z_mn) in the order (+,+), (+,-), (-,+),
// (-,-) of (min, max); the triangle with the smaller id is the outer one.
// Rules: shared vertex or centroid distance < 2h -> 7-point outer, inner =
// closed-form 1/R part (Wilton et al. 1984 / Graglia 1993) + 7-point on the
// bounded remainder (exp(-jkR) - 1)/R; distance < 4h -> 7 x 7; else 3 x 3.
// h = longest mesh edge.
#include <cmath>

#include "hps_internal.h"

namespace hps {

namespace {

const double kPi = 3.14159265358979323846;
const double kMu0 = 4.0e-7 * kPi;
const double kC0 = 299792458.0;
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);

struct Rule {
  int n;
  double b[7][3];
  double w[7];
};

Rule make_rule7() {
  Rule r;
  r.n = 7;
  const double s15 = std::sqrt(15.0);
  const double a1 = (6.0 - s15) / 21.0, w1 = (155.0 - s15) / 1200.0;
  const double a2 = (6.0 + s15) / 21.0, w2 = (155.0 + s15) / 1200.0;
  const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
  const double B[7][3] = {{1.0 / 3, 1.0 / 3, 1.0 / 3}, {b1, a1, a1}, {a1, b1, a1}, {a1, a1, b1},
                          {b2, a2, a2}, {a2, b2, a2}, {a2, a2, b2}};
  const double W[7] = {9.0 / 40.0, w1, w1, w1, w2, w2, w2};
  for (int q = 0; q < 7; ++q) {
    for (int c = 0; c < 3; ++c) r.b[q][c] = B[q][c];
    r.w[q] = W[q];
  }
  return r;
}

Rule make_rule3() {
  Rule r;
  r.n = 3;
  for (int q = 0; q < 3; ++q) {
    for (int c = 0; c < 3; ++c) r.b[q][c] = (c == q) ? 2.0 / 3.0 : 1.0 / 6.0;
    r.w[q] = 1.0 / 3.0;
  }
  return r;
}

const Rule R7 = make_rule7();
const Rule R3 = make_rule3();

inline double dot3(const double *a, const double *b) { return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2]; }

void tri_points(const Mesh &m, int32_t t, const Rule &r, double (*p)[3]) {
  const double *v0 = &m.xyz[3 * m.tri[3 * t]], *v1 = &m.xyz[3 * m.tri[3 * t + 1]],
               *v2 = &m.xyz[3 * m.tri[3 * t + 2]];
  for (int q = 0; q < r.n; ++q)
    for (int d = 0; d < 3; ++d) p[q][d] = r.b[q][0] * v0[d] + r.b[q][1] * v1[d] + r.b[q][2] * v2[d];
}

// Closed-form int_T 1/R dS' and int_T (r' - rho)/R dS' for observation point r;
// rho = projection of r on the plane of T.
void potentials(const Mesh &m, int32_t t, const double *r, double &I1, double Ir[3], double rho[3]) {
  const double *V[3] = {&m.xyz[3 * m.tri[3 * t]], &m.xyz[3 * m.tri[3 * t + 1]], &m.xyz[3 * m.tri[3 * t + 2]]};
  double e1[3], e2[3], n[3];
  for (int d = 0; d < 3; ++d) { e1[d] = V[1][d] - V[0][d]; e2[d] = V[2][d] - V[0][d]; }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nn = std::sqrt(dot3(n, n));
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  double rv[3];
  for (int d = 0; d < 3; ++d) rv[d] = r[d] - V[0][d];
  const double h = dot3(rv, n);
  const double ah = std::fabs(h);
  for (int d = 0; d < 3; ++d) rho[d] = r[d] - h * n[d];
  I1 = 0.0;
  Ir[0] = Ir[1] = Ir[2] = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double *pa = V[e], *pb = V[(e + 1) % 3];
    double s[3], u[3], da[3], db[3];
    for (int d = 0; d < 3; ++d) s[d] = pb[d] - pa[d];
    const double ls = std::sqrt(dot3(s, s));
    for (int d = 0; d < 3; ++d) s[d] /= ls;
    u[0] = s[1] * n[2] - s[2] * n[1];
    u[1] = s[2] * n[0] - s[0] * n[2];
    u[2] = s[0] * n[1] - s[1] * n[0];
    for (int d = 0; d < 3; ++d) { da[d] = pa[d] - rho[d]; db[d] = pb[d] - rho[d]; }
    const double lp = dot3(db, s), lm = dot3(da, s), t0 = dot3(da, u);
    const double R0sq = t0 * t0 + h * h;
    const double Rp = std::sqrt(lp * lp + R0sq), Rm = std::sqrt(lm * lm + R0sq);
    double F = 0.0;
    if (R0sq > 0.0)
      F = (lp + lm >= 0.0) ? std::log((Rp + lp) / (Rm + lm)) : std::log((Rm - lm) / (Rp - lp));
    double beta = 0.0;
    const double dp = R0sq + ah * Rp, dm = R0sq + ah * Rm;
    if (dp > 0.0) beta += std::atan(t0 * lp / dp);
    if (dm > 0.0) beta -= std::atan(t0 * lm / dm);
    I1 += t0 * F - ah * beta;
    const double c = 0.5 * (R0sq * F + lp * Rp - lm * Rm);
    for (int d = 0; d < 3; ++d) Ir[d] += c * u[d];
  }
}

}  // namespace

Galerkin::Galerkin(const Mesh &m, double freq_hz, bool cfie_, double alpha_) : mesh(&m), cfie(cfie_), alpha(alpha_) {
  omega = 2.0 * kPi * freq_hz;
  k = omega / kC0;
  h = m.hmax;
  cA = cplx(0.0, omega * kMu0 / 4.0);
  cPhi = cplx(0.0, -1.0 / (omega * kEps0));
}

namespace {

// (jw mu / 4) II (r - vO).(r' - vI) G - (j / (w eps)) II G over O x I (outer O).
cplx pair_integral(const Galerkin &op, int32_t O, const double *vO, int32_t I, const double *vI) {
  const Mesh &m = *op.mesh;
  const int32_t *to = &m.tri[3 * O], *ti = &m.tri[3 * I];
  bool share = false;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) share |= (to[a] == ti[b]);
  double dc[3];
  for (int d = 0; d < 3; ++d) dc[d] = m.cen[3 * O + d] - m.cen[3 * I + d];
  const double d2 = dot3(dc, dc);
  const double k = op.k;
  const double AO = m.area[O], AI = m.area[I];
  const double inv4pi = 1.0 / (4.0 * kPi);
  if (share || d2 < (2.0 * op.h) * (2.0 * op.h)) {
    double po[7][3], pi[7][3];
    tri_points(m, O, R7, po);
    tri_points(m, I, R7, pi);
    cplx acc = 0.0;
    for (int a = 0; a < 7; ++a) {
      double I1, Ir[3], rho[3];
      potentials(m, I, po[a], I1, Ir, rho);
      cplx s = I1 * inv4pi;
      cplx v[3];
      for (int d = 0; d < 3; ++d) v[d] = (Ir[d] + (rho[d] - vI[d]) * I1) * inv4pi;
      cplx gs = 0.0, gv[3] = {0.0, 0.0, 0.0};
      for (int b = 0; b < 7; ++b) {
        double dd[3];
        for (int d = 0; d < 3; ++d) dd[d] = po[a][d] - pi[b][d];
        const double R = std::sqrt(dot3(dd, dd));
        const double x = 0.5 * k * R;
        const double sinc = (x == 0.0) ? 1.0 : std::sin(x) / x;
        // (exp(-jkR) - 1) / (4 pi R) = -jk/(4 pi) sinc(kR/2) exp(-jkR/2)
        const cplx g = cplx(0.0, -k * inv4pi) * sinc * cplx(std::cos(x), -std::sin(x));
        gs += R7.w[b] * g;
        for (int d = 0; d < 3; ++d) gv[d] += R7.w[b] * (pi[b][d] - vI[d]) * g;
      }
      s += AI * gs;
      for (int d = 0; d < 3; ++d) v[d] += AI * gv[d];
      cplx dotv = 0.0;
      for (int d = 0; d < 3; ++d) dotv += (po[a][d] - vO[d]) * v[d];
      acc += R7.w[a] * (op.cA * dotv + op.cPhi * s);
    }
    return AO * acc;
  }
  const Rule &r = (d2 < (4.0 * op.h) * (4.0 * op.h)) ? R7 : R3;
  double po[7][3], pi[7][3];
  tri_points(m, O, r, po);
  tri_points(m, I, r, pi);
  cplx acc = 0.0;
  for (int a = 0; a < r.n; ++a) {
    double ro[3];
    for (int d = 0; d < 3; ++d) ro[d] = po[a][d] - vO[d];
    cplx inner = 0.0;
    for (int b = 0; b < r.n; ++b) {
      double dd[3], ri[3];
      for (int d = 0; d < 3; ++d) { dd[d] = po[a][d] - pi[b][d]; ri[d] = pi[b][d] - vI[d]; }
      const double R = std::sqrt(dot3(dd, dd));
      const cplx G = cplx(std::cos(k * R), -std::sin(k * R)) * (inv4pi / R);
      inner += r.w[b] * G * (op.cA * dot3(ro, ri) + op.cPhi);
    }
    acc += r.w[a] * inner;
  }
  return AO * AI * acc;
}

}  // namespace

cplx Galerkin::efie_entry(int64_t m_, int64_t n_) const {
  const Mesh &m = *mesh;
  const int64_t a = m_ < n_ ? m_ : n_, b = m_ < n_ ? n_ : m_;
  const int32_t ta[2] = {m.tp[a], m.tm[a]}, tb[2] = {m.tp[b], m.tm[b]};
  const int32_t va[2] = {m.vp[a], m.vm[a]}, vb[2] = {m.vp[b], m.vm[b]};
  const double sg[2] = {1.0, -1.0};
  cplx z = 0.0;
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) {
      const int32_t P = ta[p], Q = tb[q];
      const double *vP = &m.xyz[3 * va[p]], *vQ = &m.xyz[3 * vb[q]];
      const cplx I = (P <= Q) ? pair_integral(*this, P, vP, Q, vQ) : pair_integral(*this, Q, vQ, P, vP);
      z += (sg[p] * sg[q] * m.len[a] * m.len[b] / (m.area[P] * m.area[Q])) * I;
    }
  return z;
}

namespace {

// int_T (r - r') / R^3 dS' for observation point r: the in-plane part is the
// divergence theorem on grad'_s (1/R) = (rho - r') / R^3, sum_i u_i F_i, the
// normal part sign(d) sum_i beta_i (the arctangent terms of potentials()).
void grad_potential(const Mesh &m, int32_t t, const double *r, double out[3]) {
  const double *V[3] = {&m.xyz[3 * m.tri[3 * t]], &m.xyz[3 * m.tri[3 * t + 1]], &m.xyz[3 * m.tri[3 * t + 2]]};
  double e1[3], e2[3], n[3];
  for (int d = 0; d < 3; ++d) { e1[d] = V[1][d] - V[0][d]; e2[d] = V[2][d] - V[0][d]; }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double nn = std::sqrt(dot3(n, n));
  for (int d = 0; d < 3; ++d) n[d] /= nn;
  double rv[3], rho[3];
  for (int d = 0; d < 3; ++d) rv[d] = r[d] - V[0][d];
  const double h = dot3(rv, n), ah = std::fabs(h);
  for (int d = 0; d < 3; ++d) rho[d] = r[d] - h * n[d];
  out[0] = out[1] = out[2] = 0.0;
  double bsum = 0.0;
  for (int e = 0; e < 3; ++e) {
    const double *pa = V[e], *pb = V[(e + 1) % 3];
    double sv[3], u[3], da[3], db[3];
    for (int d = 0; d < 3; ++d) sv[d] = pb[d] - pa[d];
    const double ls = std::sqrt(dot3(sv, sv));
    for (int d = 0; d < 3; ++d) sv[d] /= ls;
    u[0] = sv[1] * n[2] - sv[2] * n[1];
    u[1] = sv[2] * n[0] - sv[0] * n[2];
    u[2] = sv[0] * n[1] - sv[1] * n[0];
    for (int d = 0; d < 3; ++d) { da[d] = pa[d] - rho[d]; db[d] = pb[d] - rho[d]; }
    const double lp = dot3(db, sv), lm = dot3(da, sv), t0 = dot3(da, u);
    const double R0sq = t0 * t0 + h * h;
    const double Rp = std::sqrt(lp * lp + R0sq), Rm = std::sqrt(lm * lm + R0sq);
    double F = 0.0;
    if (R0sq > 0.0)
      F = (lp + lm >= 0.0) ? std::log((Rp + lp) / (Rm + lm)) : std::log((Rm - lm) / (Rp - lp));
    double beta = 0.0;
    const double dp = R0sq + ah * Rp, dm = R0sq + ah * Rm;
    if (dp > 0.0) beta += std::atan(t0 * lp / dp);
    if (dm > 0.0) beta -= std::atan(t0 * lm / dm);
    for (int d = 0; d < 3; ++d) out[d] += u[d] * F;
    bsum += beta;
  }
  const double sg = (h > 0.0) ? 1.0 : (h < 0.0 ? -1.0 : 0.0);
  for (int d = 0; d < 3; ++d) out[d] += n[d] * sg * bsum;
}

// MFIE kernel (1 + jkR) exp(-jkR) / (4 pi R^3) (eq. 7 times 1/R) and its part
// without the static 1/(4 pi R^3).
inline void mfie_kernel(double k, double R, cplx &g, cplx &gdyn) {
  const double x = k * R, c = std::cos(x), s = std::sin(x);
  const cplx num(c - 1.0 + x * s, x * c - s);     // (1 + jx) e^{-jx} - 1
  const double den = 4.0 * kPi * R * R * R;
  gdyn = num / den;
  g = (1.0 + num) / den;
}

// int_P (r - vP) . [n_P x ((r - vQ) x W_Q(r))] dS with
// W_Q(r) = int_Q (r - r') g(R) dS', for P != Q; written as
// (a.b)(n.W) - (a.W)(n.b), a = r - vP, b = r - vQ.  Rules as for the EFIE:
// touching or < 2h: 7-point outer, closed-form static part + 7 points on the
// remainder; < 4h: 7 x 7; else 3 x 3.
cplx mfie_pair(const Galerkin &op, int32_t P, const double *vP, int32_t Q, const double *vQ) {
  const Mesh &m = *op.mesh;
  const int32_t *tp = &m.tri[3 * P], *tq = &m.tri[3 * Q];
  bool share = false;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) share |= (tp[a] == tq[b]);
  double dc[3];
  for (int d = 0; d < 3; ++d) dc[d] = m.cen[3 * P + d] - m.cen[3 * Q + d];
  const double d2 = dot3(dc, dc);
  const int rule = (share || d2 < (2.0 * op.h) * (2.0 * op.h)) ? 0 : (d2 < (4.0 * op.h) * (4.0 * op.h) ? 1 : 2);
  const Rule &rr = rule == 2 ? R3 : R7;
  double po[7][3], pi[7][3];
  tri_points(m, P, rr, po);
  tri_points(m, Q, rr, pi);
  const double *nP = &m.nrm[3 * P];
  const double AQ = m.area[Q];
  cplx acc = 0.0;
  for (int a = 0; a < rr.n; ++a) {
    cplx W[3] = {0.0, 0.0, 0.0};
    for (int b = 0; b < rr.n; ++b) {
      double dd[3];
      for (int d = 0; d < 3; ++d) dd[d] = po[a][d] - pi[b][d];
      const double R = std::sqrt(dot3(dd, dd));
      cplx g, gdyn;
      mfie_kernel(op.k, R, g, gdyn);
      const cplx f = rr.w[b] * AQ * (rule == 0 ? gdyn : g);
      for (int d = 0; d < 3; ++d) W[d] += f * dd[d];
    }
    if (rule == 0) {
      double V[3];
      grad_potential(m, Q, po[a], V);
      for (int d = 0; d < 3; ++d) W[d] += V[d] / (4.0 * kPi);
    }
    double am[3], bn[3];
    for (int d = 0; d < 3; ++d) { am[d] = po[a][d] - vP[d]; bn[d] = po[a][d] - vQ[d]; }
    const cplx nW = (nP[0] * W[0] + nP[1] * W[1]) + nP[2] * W[2];
    const cplx aW = (am[0] * W[0] + am[1] * W[1]) + am[2] * W[2];
    acc += rr.w[a] * (dot3(am, bn) * nW - aW * dot3(nP, bn));
  }
  return m.area[P] * acc;
}

}  // namespace

// MFIE (eqs. 6-7) tested with f_m: 1/2 <f_m, f_n> - <f_m, n x int f_n x grad' G>,
// summed over the triangle pairs (+,+), (+,-), (-,+), (-,-) of (m, n); on one
// flat triangle the integral term vanishes.
cplx Galerkin::mfie_entry(int64_t m_, int64_t n_) const {
  const Mesh &m = *mesh;
  const int32_t tm_[2] = {m.tp[m_], m.tm[m_]}, tn_[2] = {m.tp[n_], m.tm[n_]};
  const int32_t vm_[2] = {m.vp[m_], m.vm[m_]}, vn_[2] = {m.vp[n_], m.vm[n_]};
  const double sg[2] = {1.0, -1.0};
  cplx z = 0.0;
  for (int p = 0; p < 2; ++p)
    for (int q = 0; q < 2; ++q) {
      const int32_t P = tm_[p], Q = tn_[q];
      const double *vP = &m.xyz[3 * vm_[p]], *vQ = &m.xyz[3 * vn_[q]];
      const double c = sg[p] * sg[q] * m.len[m_] * m.len[n_] / (4.0 * m.area[P] * m.area[Q]);
      cplx v;
      if (P == Q) {
        double pts[7][3];
        tri_points(m, P, R7, pts);
        double acc = 0.0;
        for (int a = 0; a < 7; ++a) {
          double am[3], bn[3];
          for (int d = 0; d < 3; ++d) { am[d] = pts[a][d] - vP[d]; bn[d] = pts[a][d] - vQ[d]; }
          acc += R7.w[a] * dot3(am, bn);
        }
        v = 0.5 * m.area[P] * acc;
      } else {
        v = -mfie_pair(*this, P, vP, Q, vQ);
      }
      z += c * v;
    }
  return z;
}

cplx Galerkin::entry(int64_t m_, int64_t n_) const {
  if (!cfie) return efie_entry(m_, n_);
  cplx z = alpha * efie_entry(m_, n_);
  if (alpha != 1.0) z += (kMu0 * kC0) * (1.0 - alpha) * mfie_entry(m_, n_);
  return z;
}

void Galerkin::block(const int64_t *rows, int64_t nr, const int64_t *cols, int64_t nc, cplx *out) const {
  for (int64_t i = 0; i < nr; ++i)
    for (int64_t j = 0; j < nc; ++j) out[i * nc + j] = entry(rows[i], cols[j]);
}

}  // namespace hps
