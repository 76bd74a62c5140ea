// Operator and load of 2D elasticity on a quadrilateral domain in QTT format (Alg. 1 of the
// paper in full, Sec. 5.1-5.3).
//
// The domain is the bilinear image x(s, t) of the unit square with corners P00, P10, P01,
// P11; node (i, j) of the 2^d x 2^d grid sits at x(i / (2^d - 1), j / (2^d - 1)).  Element
// m = (i, j) has corners x(i + cx, j + cy).  As Alg. 1 states, the element Jacobian J_m and
// det J_m are taken at the element centre xi = (0, 0); they are affine / bilinear functions
// of (i, j) (eq. affinejacs).  With J frozen, the element stiffness separates into
//
//   K_m[(a, c1), (b, c2)] = sum_{g, h} G_{a g b h}(m) Wx_{gh}[c1x][c2x] Wy_{gh}[c1y][c2y],
//   G_{a g b h}(m) = sum_{al, be} C_{a al b be} (J_m^-1)_{g al} (J_m^-1)_{h be} det J_m,
//
// with Wx, Wy the 1D reference integrals (value or derivative of the test / trial corner
// function on each axis).  The 16 coefficient fields G_{a g b h} over the element grid are
// sampled and compressed to QTT (TT-SVD of the sampled field at 1e-14: the component-wise
// inverse of det J that the paper approximates by TT-cross is exact up to that rounding
// here), one TT per derivative pair (g, h) carrying (a, b) as a last core.  The global
// operator places each element contribution at the node pair (m + c1, m + c2): per axis a
// carry automaton F_W[p, q, m] = sum_{c1, c2} W[c1][c2] [p = m + c1][q = m + c2] (MSB-first
// cores, bond state = the two carries), the corner-pair sum of the paper done exactly by
// the automaton.  Clamped sides mask p and q inside F (symmetric elimination), then
// alpha (I - P) is added; the four (g, h) terms are summed and rounded at 1e-14.  The mass
// operator is built the same way from the field det J_m; the load is P M f0 plus side
// tractions.
#include <algorithm>
#include <array>
#include <cmath>
#include <vector>

#include "assembly.hpp"
#include "common.hpp"
#include "hostla.hpp"

namespace tnfem {
namespace {

// A TT with fused physical indices; for operators the level mode is (p, q) -> p * 4 + q.
using Cores = std::vector<TTCore>;

// TT-SVD of a dense array with the given modes (row-major, last mode fastest) at relative
// accuracy eps.
Cores tt_svd_dense(std::vector<double> a, const std::vector<int>& modes, double eps) {
  const int K = (int)modes.size();
  double nrm = 0.0;
  for (double v : a) nrm += v * v;
  nrm = std::sqrt(nrm);
  const double delta = eps * nrm / std::sqrt((double)std::max(K - 1, 1));
  Cores out;
  int r = 1;
  size_t cols = a.size();
  for (int k = 0; k < K - 1; ++k) {
    const int m = r * modes[k];
    cols /= modes[k];
    std::vector<double> U, S, Vt;
    hostla::svd(m, (int)cols, a.data(), U, S, Vt);
    const int c = (int)S.size();
    double tail = 0.0;
    int rk = c;
    for (int j = c - 1; j >= 1; --j) {
      if (tail + S[j] * S[j] <= delta * delta) {
        tail += S[j] * S[j];
        rk = j;
      } else {
        break;
      }
    }
    TTCore core;
    core.rl = r;
    core.n = modes[k];
    core.rr = rk;
    core.data.resize((size_t)m * rk);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < rk; ++j) core.data[(size_t)i * rk + j] = U[(size_t)i * c + j];
    out.push_back(core);
    std::vector<double> rest((size_t)rk * cols);
    for (int i = 0; i < rk; ++i)
      for (size_t j = 0; j < cols; ++j) rest[i * cols + j] = S[i] * Vt[i * cols + j];
    a.swap(rest);
    r = rk;
  }
  TTCore last;
  last.rl = r;
  last.n = modes[K - 1];
  last.rr = 1;
  last.data = a;
  out.push_back(last);
  return out;
}

// 1D node mask 1 - c0 [p = 0] - c1 [p = 2^d - 1] as a QTT vector (exact rank <= 3).
Cores node_mask(int d, bool clamp0, bool clamp1) {
  std::vector<double> m((size_t)1 << d, 1.0);
  if (clamp0) m.front() = 0.0;
  if (clamp1) m.back() = 0.0;
  return vector_qtt(m, d);
}

// F[p, q, m] * M[p] (on_p) or * M[q]: the product with a QTT vector M on one node index.
Cores mask_index(const Cores& F, const Cores& M, bool on_p) {
  const int d = (int)F.size();
  Cores G(d);
  for (int l = 0; l < d; ++l) {
    const TTCore &f = F[l], &mk = M[l];
    TTCore g;
    g.rl = f.rl * mk.rl;
    g.rr = f.rr * mk.rr;
    g.n = 8;
    g.data.assign((size_t)g.rl * 8 * g.rr, 0.0);
    for (int fa = 0; fa < f.rl; ++fa)
      for (int ma = 0; ma < mk.rl; ++ma)
        for (int e = 0; e < 8; ++e) {
          const int bit = on_p ? (e >> 2) & 1 : (e >> 1) & 1;
          for (int fb = 0; fb < f.rr; ++fb) {
            const double fv = f.data[((size_t)fa * 8 + e) * f.rr + fb];
            if (fv == 0.0) continue;
            for (int mb = 0; mb < mk.rr; ++mb)
              g.data[(((size_t)fa * mk.rl + ma) * 8 + e) * g.rr + fb * mk.rr + mb] +=
                  fv * mk.data[((size_t)ma * 2 + bit) * mk.rr + mb];
          }
        }
    G[l] = g;
  }
  tt_round_host(G, 1e-15, 1 << 30);
  return G;
}

// 1D element-to-node automaton F[p, q, m] = sum_{c1, c2} W[c1][c2] [p = m + c1][q = m + c2]
// on 2^d nodes / elements: d cores [s][(p * 2 + q) * 2 + m][s'] with the bond state s =
// (carry of p, carry of q) handed up from the less significant levels, most significant
// level first; then the node masks of clamped ends on p (and on q when mask_q).
Cores axis_automaton(int d, const double W[2][2], bool clamp0, bool clamp1, bool mask_q) {
  Cores F(d);
  for (int l = 0; l < d; ++l) {
    TTCore c;
    c.rl = l == 0 ? 1 : 4;
    c.rr = l == d - 1 ? 1 : 4;
    c.n = 8;
    c.data.assign((size_t)c.rl * 8 * c.rr, 0.0);
    for (int m = 0; m < 2; ++m) {
      // carries coming in: the corner offsets (weighted) at the least significant level,
      // the right bond state above it
      for (int si = 0; si < 4; ++si) {
        const int ci = si >> 1, di = si & 1;
        const double w = l == d - 1 ? W[ci][di] : 1.0;
        if (w == 0.0) continue;
        const int p = (m + ci) & 1, q = (m + di) & 1, so = ((m + ci) >> 1) * 2 + ((m + di) >> 1);
        if (l == 0 && so != 0) continue;  // no overflow out of the most significant level
        const int row = l == 0 ? 0 : so, col = l == d - 1 ? 0 : si;
        c.data[((size_t)row * 8 + (p * 2 + q) * 2 + m) * c.rr + col] += w;
      }
    }
    F[l] = c;
  }
  if (clamp0 || clamp1) {
    const Cores M = node_mask(d, clamp0, clamp1);
    F = mask_index(F, M, true);
    if (mask_q) F = mask_index(F, M, false);
  }
  return F;
}

// Diagonal operator diag(v) (level mode p * 4 + q, p = q) of a vector TT v in the solution
// layout; the component core is diag(v_comp).
Cores diag_operator(const Cores& v) {
  const int K = (int)v.size();
  Cores o(K);
  for (int k = 0; k < K; ++k) {
    const int nm = v[k].n;
    TTCore c;
    c.rl = v[k].rl;
    c.rr = v[k].rr;
    c.n = nm * nm;
    c.data.assign((size_t)c.rl * c.n * c.rr, 0.0);
    for (int a = 0; a < c.rl; ++a)
      for (int i = 0; i < nm; ++i)
        for (int b = 0; b < c.rr; ++b)
          c.data[((size_t)a * c.n + i * nm + i) * c.rr + b] = v[k].data[((size_t)a * nm + i) * c.rr + b];
    o[k] = c;
  }
  return o;
}

// Level cores of sum_m G(m) F_x[p_x, q_x, m_x] F_y[p_y, q_y, m_y] as an operator TT with
// level mode (p, q) = ((p_x p_y), (q_x q_y)) -> p * 4 + q, and the field's last core (the
// component pair (a, b)) as the component core (mode a * 2 + b).
Cores stencil_operator(const Cores& Fx, const Cores& Fy, const Cores& G) {
  const int d = (int)Fx.size();
  Cores out(d + 1);
  for (int l = 0; l < d; ++l) {
    const TTCore &fx = Fx[l], &fy = Fy[l], &g = G[l];
    TTCore o;
    o.rl = g.rl * fx.rl * fy.rl;
    o.rr = g.rr * fx.rr * fy.rr;
    o.n = 16;
    o.data.assign((size_t)o.rl * 16 * o.rr, 0.0);
    for (int ga = 0; ga < g.rl; ++ga)
      for (int xa = 0; xa < fx.rl; ++xa)
        for (int ya = 0; ya < fy.rl; ++ya)
          for (int gb = 0; gb < g.rr; ++gb)
            for (int xb = 0; xb < fx.rr; ++xb)
              for (int yb = 0; yb < fy.rr; ++yb)
                for (int mx = 0; mx < 2; ++mx)
                  for (int my = 0; my < 2; ++my) {
                    const double gv = g.data[((size_t)ga * 4 + mx * 2 + my) * g.rr + gb];
                    if (gv == 0.0) continue;
                    for (int pqx = 0; pqx < 4; ++pqx) {
                      const double xv = fx.data[((size_t)xa * 8 + pqx * 2 + mx) * fx.rr + xb];
                      if (xv == 0.0) continue;
                      for (int pqy = 0; pqy < 4; ++pqy) {
                        const double yv = fy.data[((size_t)ya * 8 + pqy * 2 + my) * fy.rr + yb];
                        if (yv == 0.0) continue;
                        const int p = (pqx >> 1) * 2 + (pqy >> 1), q = (pqx & 1) * 2 + (pqy & 1);
                        const size_t row = ((size_t)ga * fx.rl + xa) * fy.rl + ya;
                        const size_t col = ((size_t)gb * fx.rr + xb) * fy.rr + yb;
                        o.data[(row * 16 + p * 4 + q) * o.rr + col] += gv * xv * yv;
                      }
                    }
                  }
    out[l] = o;
  }
  out[d] = G[d];  // [r][a * 2 + b][1]: the component core of mode (a, b)
  return out;
}

// Operator TT (level mode 16, component mode 4) -> MPO cores as nonzero lists.
std::vector<MpoCore> to_mpo(const Cores& T) {
  std::vector<MpoCore> A;
  const int K = (int)T.size();
  for (int k = 0; k < K; ++k) {
    const TTCore& c = T[k];
    const int nm = k < K - 1 ? 4 : 2;
    MpoCore m;
    m.Rl = c.rl;
    m.Rr = c.rr;
    m.n = nm;
    for (int a = 0; a < c.rl; ++a)
      for (int i = 0; i < nm; ++i)
        for (int j = 0; j < nm; ++j)
          for (int b = 0; b < c.rr; ++b) {
            const double v = c.data[((size_t)a * nm * nm + i * nm + j) * c.rr + b];
            if (v != 0.0) m.add(a, i, j, b, v);
          }
    A.push_back(m);
  }
  return A;
}

// y = A x for an operator TT (level mode p * 4 + q) and a vector TT of the same layout.
Cores apply_operator(const Cores& A, const Cores& x) {
  const int K = (int)A.size();
  Cores y(K);
  for (int k = 0; k < K; ++k) {
    const TTCore &a = A[k], &v = x[k];
    const int nm = k < K - 1 ? 4 : 2;
    TTCore o;
    o.rl = a.rl * v.rl;
    o.rr = a.rr * v.rr;
    o.n = nm;
    o.data.assign((size_t)o.rl * nm * o.rr, 0.0);
    for (int ra = 0; ra < a.rl; ++ra)
      for (int rv = 0; rv < v.rl; ++rv)
        for (int p = 0; p < nm; ++p)
          for (int q = 0; q < nm; ++q)
            for (int sa = 0; sa < a.rr; ++sa) {
              const double av = a.data[((size_t)ra * nm * nm + p * nm + q) * a.rr + sa];
              if (av == 0.0) continue;
              for (int sv = 0; sv < v.rr; ++sv)
                o.data[(((size_t)ra * v.rl + rv) * nm + p) * o.rr + sa * v.rr + sv] +=
                    av * v.data[((size_t)rv * nm + q) * v.rr + sv];
            }
    y[k] = o;
  }
  return y;
}

}  // namespace

Assembled assemble_quad(const tnfem_problem_desc& desc) {
  const int D = desc.dim, d = desc.level;
  TNFEM_REQUIRE(D == 2, "a quadrilateral domain is 2D");
  TNFEM_REQUIRE(d >= 2 && d <= 8, "level must be in [2, 8] on a quadrilateral domain (got %d)", d);
  TNFEM_REQUIRE(desc.layer_E == nullptr, "layer_E does not combine with a quadrilateral domain");
  const int nel = (1 << d) - 1;
  if (desc.elem_weight) {
    TNFEM_REQUIRE(desc.n_elem_weight == nel * nel, "elem_weight must hold (2^d - 1)^2 = %d values", nel * nel);
    for (int e = 0; e < nel * nel; ++e)
      TNFEM_REQUIRE(desc.elem_weight[e] > 0 && std::isfinite(desc.elem_weight[e]), "elem_weight must be positive");
  }
  TNFEM_REQUIRE(!desc.has_manufactured, "the manufactured load is defined on the unit box only");
  TNFEM_REQUIRE(desc.E > 0 && std::isfinite(desc.E), "E must be positive");
  TNFEM_REQUIRE(desc.nu > -1.0 && desc.nu < 0.5, "nu must be in (-1, 0.5)");
  TNFEM_REQUIRE(!(desc.plane_stress && desc.has_stiffness), "plane_stress does not combine with a stiffness matrix");
  TNFEM_REQUIRE((desc.clamp_mask >> 4) == 0, "clamp_mask names a face beyond dim");
  TNFEM_REQUIRE(desc.n_tractions >= 0 && desc.n_tractions <= 4, "n_tractions must be in [0, 4]");
  for (int c = 0; c < 4; ++c)
    for (int k = 0; k < 2; ++k) TNFEM_REQUIRE(std::isfinite(desc.quad[c][k]), "quad corners must be finite");
  const int n = 1 << d;
  double lam = desc.E * desc.nu / ((1 + desc.nu) * (1 - 2 * desc.nu));
  double mu = desc.E / (2 * (1 + desc.nu));
  if (desc.plane_stress) lam = 2 * lam * mu / (lam + 2 * mu);
  const std::vector<double> Ct = stiffness_tensor(desc, 2, lam, mu);
  auto Cq = [&](int i, int a, int j, int b) { return Ct[((i * 2 + a) * 2 + j) * 2 + b]; };
  const double alpha = std::max(Cq(0, 0, 0, 0), Cq(1, 1, 1, 1));  // h^(D-2) = 1 in 2D

  Assembled out;
  out.D = 2;
  out.d = d;
  out.lam = lam;
  out.mu = mu;
  out.alpha = alpha;

  // node coordinates of the bilinear map
  const double(*P)[2] = desc.quad;  // P00, P10, P01, P11
  auto X = [&](int i, int j, int k) {
    const double s = (double)i / (n - 1), t = (double)j / (n - 1);
    return P[0][k] * (1 - s) * (1 - t) + P[1][k] * s * (1 - t) + P[2][k] * (1 - s) * t + P[3][k] * s * t;
  };

  // coefficient fields over the element grid (QTT order: level mode (i bit) * 2 + (j bit)),
  // the element index 2^d - 1 void; per (g, h) an array [level modes][(a, b)]
  const size_t ne = (size_t)n * n;
  std::vector<std::vector<double>> Gf(4, std::vector<double>(ne * 4, 0.0));
  std::vector<double> detf(ne, 0.0);
  for (int i = 0; i + 1 < n; ++i)
    for (int j = 0; j + 1 < n; ++j) {
      // J0[k][g] = sum_c x_c[k] d phi_c / d xi_g at xi = 0 = (1/4) sum_c sign_{c,g} x_c[k]
      double J[2][2];
      for (int k = 0; k < 2; ++k) {
        J[k][0] = 0.25 * (X(i + 1, j, k) + X(i + 1, j + 1, k) - X(i, j, k) - X(i, j + 1, k));
        J[k][1] = 0.25 * (X(i, j + 1, k) + X(i + 1, j + 1, k) - X(i, j, k) - X(i + 1, j, k));
      }
      const double det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      TNFEM_REQUIRE(det > 0.0, "the quadrilateral must be convex with corners P00, P10, P01, P11 counterclockwise "
                               "(element (%d, %d) has det J <= 0)", i, j);
      const double inv[2][2] = {{J[1][1] / det, -J[0][1] / det}, {-J[1][0] / det, J[0][0] / det}};
      size_t q = 0;
      for (int l = 0; l < d; ++l) q = q * 4 + (((i >> (d - 1 - l)) & 1) * 2 + ((j >> (d - 1 - l)) & 1));
      detf[q] = det;
      for (int g = 0; g < 2; ++g)
        for (int h = 0; h < 2; ++h)
          for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
              double v = 0.0;
              for (int al = 0; al < 2; ++al)
                for (int be = 0; be < 2; ++be) v += Cq(a, al, b, be) * inv[g][al] * inv[h][be];
              Gf[g * 2 + h][q * 4 + a * 2 + b] = v * det * (desc.elem_weight ? desc.elem_weight[i * nel + j] : 1.0);
            }
    }
  std::vector<int> fmodes(d, 4);
  fmodes.push_back(4);

  // 1D reference integrals on [-1, 1] of the corner functions (0: (1 - xi)/2, 1: (1 + xi)/2)
  const double V[2][2] = {{2.0 / 3, 1.0 / 3}, {1.0 / 3, 2.0 / 3}};  // value, value
  const double Dd[2][2] = {{0.5, -0.5}, {-0.5, 0.5}};              // derivative, derivative
  const double DV[2][2] = {{-0.5, -0.5}, {0.5, 0.5}};              // derivative (test), value
  const double VD[2][2] = {{-0.5, 0.5}, {-0.5, 0.5}};              // value (test), derivative
  const bool c0[2] = {(desc.clamp_mask & 1u) != 0, (desc.clamp_mask & 4u) != 0};
  const bool c1[2] = {(desc.clamp_mask & 2u) != 0, (desc.clamp_mask & 8u) != 0};
  auto weight = [&](int axis, int g, int h) -> const double(*)[2] {
    const bool dt = g == axis, dr = h == axis;
    return dt ? (dr ? Dd : DV) : (dr ? VD : V);
  };

  // stiffness: sum over derivative pairs (g, h)
  Cores total;
  for (int g = 0; g < 2; ++g)
    for (int h = 0; h < 2; ++h) {
      Cores G = tt_svd_dense(Gf[g * 2 + h], fmodes, 1e-14);
      Cores Fx = axis_automaton(d, weight(0, g, h), c0[0], c1[0], true);
      Cores Fy = axis_automaton(d, weight(1, g, h), c0[1], c1[1], true);
      Cores term = stencil_operator(Fx, Fy, G);
      tt_round_host(term, 1e-14, 1 << 30);
      if (total.empty()) {
        total = term;
      } else {
        total = tt_sum(total, term);
        tt_round_host(total, 1e-14, 1 << 30);
      }
    }
  // alpha (I - P) with P the mask of the dofs not clamped: diag(alpha (1 - mask)) (x) I_2
  const bool any = c0[0] || c1[0] || c0[1] || c1[1];
  if (any) {
    const Cores mx = node_mask(d, c0[0], c1[0]), my = node_mask(d, c0[1], c1[1]);
    Cores mask = kron_vector_levels({mx, my});
    TTCore comp;
    comp.n = 2;
    comp.data = {1.0, 1.0};
    mask.push_back(comp);
    Cores ones(d + 1);
    for (int l = 0; l < d; ++l) {
      ones[l].n = 4;
      ones[l].data.assign(4, 1.0);
    }
    ones[d].n = 2;
    ones[d].data = {alpha, alpha};
    for (double& v : mask[0].data) v *= -alpha;
    Cores fixed = tt_sum(ones, mask);  // alpha (1 - mask) on every component
    tt_round_host(fixed, 1e-15, 1 << 30);
    total = tt_sum(total, diag_operator(fixed));
  }
  tt_round_host(total, 1e-14, 1 << 30);
  out.A = to_mpo(total);

  // load: P M f0 (constant body force and / or nodal TT) plus side tractions
  Cores b;
  auto add = [&](Cores t) {
    if (b.empty()) {
      b = std::move(t);
    } else {
      b = tt_sum(b, t);
      tt_round_host(b, 1e-14, 1 << 30);
    }
  };
  const bool f0 = desc.f0_cores != nullptr;
  if (desc.has_body_force || f0) {
    // P M: the mass stencil with the field det J_m (component identity), p masked
    std::vector<double> mf(ne * 4, 0.0);
    for (size_t q = 0; q < ne; ++q) mf[q * 4 + 0] = mf[q * 4 + 3] = detf[q];
    Cores Gm = tt_svd_dense(mf, fmodes, 1e-14);
    Cores Mop = stencil_operator(axis_automaton(d, V, c0[0], c1[0], false), axis_automaton(d, V, c0[1], c1[1], false), Gm);
    tt_round_host(Mop, 1e-14, 1 << 30);
    if (desc.has_body_force) {
      Cores f(d + 1);
      for (int l = 0; l < d; ++l) {
        f[l].n = 4;
        f[l].data.assign(4, 1.0);
      }
      f[d].n = 2;
      f[d].data = {desc.body_force[0], desc.body_force[1]};
      Cores y = apply_operator(Mop, f);
      tt_round_host(y, 1e-14, 1 << 30);
      add(y);
    }
    if (f0) {
      f0_doubles(desc);  // validates the ranks before any core is read
      Cores x(d + 1);
      size_t off = 0;
      for (int k = 0; k <= d; ++k) {
        x[k].rl = desc.f0_ranks[k];
        x[k].rr = desc.f0_ranks[k + 1];
        x[k].n = k < d ? 4 : 2;
        const size_t sz = (size_t)x[k].rl * x[k].n * x[k].rr;
        x[k].data.assign(desc.f0_cores + off, desc.f0_cores + off + sz);
        for (double v : x[k].data) TNFEM_REQUIRE(std::isfinite(v), "f0 holds a non-finite value");
        off += sz;
      }
      Cores y = apply_operator(Mop, x);
      tt_round_host(y, 1e-14, 1 << 30);
      add(y);
    }
  }
  for (int q = 0; q < desc.n_tractions; ++q) {
    const int face = desc.traction_face[q];
    TNFEM_REQUIRE(face >= 0 && face < 4, "traction face %d out of range", face);
    const int ax = face / 2, side = face % 2;
    // the side's end corners (P00, P10, P01, P11 = 0, 1, 2, 3) and its node spacing
    static const int ends[4][2] = {{0, 2}, {1, 3}, {0, 1}, {2, 3}};
    const double* A0 = P[ends[face][0]];
    const double* A1 = P[ends[face][1]];
    const double L = std::hypot(A1[0] - A0[0], A1[1] - A0[1]);
    const double hs = L / (n - 1);
    std::vector<std::vector<TTCore>> axes;
    for (int a = 0; a < 2; ++a) {
      std::vector<double> v(n, 0.0);
      if (a == ax) {
        v[side ? n - 1 : 0] = 1.0;
      } else {
        std::fill(v.begin(), v.end(), hs);
        v.front() = v.back() = 0.5 * hs;
      }
      if (c0[a]) v.front() = 0.0;
      if (c1[a]) v.back() = 0.0;
      axes.push_back(vector_qtt(v, d));
    }
    Cores t = kron_vector_levels(axes);
    TTCore comp;
    comp.n = 2;
    comp.data = {desc.traction[q][0], desc.traction[q][1]};
    t.push_back(comp);
    add(t);
  }
  if (b.empty()) {
    b.resize(d + 1);
    for (int l = 0; l <= d; ++l) {
      b[l].n = l < d ? 4 : 2;
      b[l].data.assign(b[l].n, 0.0);
    }
  }
  out.b = b;
  return out;
}

}  // namespace tnfem
