// Host assembly of the QTT stiffness operator and load vector.
//
// On a Cartesian box with constant Jacobians the element-by-element assembly of
// eq. elassembly factorises over axes.  For test component a / trial component b
//   K_ab = lambda D_ab + mu D_ba + mu delta_ab sum_c D_cc,
// where D_ab is a Kronecker product of 1D Q1 integrals: S (phi' phi') on axis a
// and M (phi phi) elsewhere when a == b; G (phi' phi) on a, G^T on b, M elsewhere
// otherwise.  Every 1D factor on 2^d nodes is a combination of nine matrices:
// I, the upper shift J, J^T and six corner units (E00, Ell, E01, E10, E_{l,l-1},
// E_{l-1,l}).  In QTT format (levels most significant first, Sec. 4) all nine
// are read by one five-state carry automaton per axis:
//   EQ: row and column prefixes equal;  C: column prefix = row prefix + 1 with
//   the carry still to be absorbed (for J);  B: the same for J^T;
//   Z: both prefixes all zeros;  O: both prefixes all ones.
// A level core of the D-dimensional operator is the Kronecker product of the
// axes' automaton steps (5^D states), the last level core maps the final states
// to the "atoms" D_ab (and the boundary-condition atoms), and the component core
// combines atoms with the material constants.  The result is exact (no rounding)
// and its middle cores are 0/1 matrices with one nonzero per (input state,
// mode) pair -- the structure the device contraction kernels exploit.
// Clamped faces: A_bc = P A P + alpha (I - P), alpha = max_i C_iiii h_x^(D-2) (lambda + 2 mu when isotropic),
// with P the Kronecker product of 1D masks (symmetric elimination).
#include "assembly.hpp"

#include <algorithm>
#include <array>
#include <cmath>

#include "common.hpp"
#include "hostla.hpp"

namespace tnfem {

std::vector<double> MpoCore::dense() const {
  std::vector<double> out((size_t)Rl * n * n * Rr, 0.0);
  for (size_t t = 0; t < v.size(); ++t)
    out[(((size_t)b[t] * n + io[t]) * n + ii[t]) * Rr + e[t]] += v[t];
  return out;
}

namespace {

enum Basis { I_ = 0, J_, JT_, E00_, ELL_, E01_, E10_, ELLM_, ELML_, LZ_, U_, NBASIS };
// Layered axis only: LZ, the equal-prefix path whose bits below the layer level
// are all zero; U, an unweighted copy of the equal-prefix path (for the
// boundary atoms, which are not element sums).
enum State { EQ = 0, C = 1, B = 2, Z = 3, O = 4, NSTATE = 5, LZ = 5, U = 6 };

struct Factor {
  std::array<double, NBASIS> f{};
};

Factor masked(Factor F, bool clamp0, bool clamp1) {
  // P F P with P = I - [clamp0] E00 - [clamp1] Ell: zero the first/last row and column.
  if (clamp0) {
    F.f[E00_] = -F.f[I_];
    F.f[E01_] = -F.f[J_];
    F.f[E10_] = -F.f[JT_];
  }
  if (clamp1) {
    F.f[ELL_] = -F.f[I_];
    F.f[ELLM_] = -F.f[JT_];
    F.f[ELML_] = -F.f[J_];
  }
  return F;
}

// Per-axis automaton entries: (state in, out bit, in bit, state out, value).
struct Step {
  int s, io, ii, t;
  double v;
};

std::vector<Step> first_steps() {
  return {{0, 0, 0, EQ, 1}, {0, 1, 1, EQ, 1}, {0, 0, 1, C, 1},
          {0, 1, 0, B, 1},  {0, 0, 0, Z, 1},  {0, 1, 1, O, 1}};
}

std::vector<Step> middle_steps() {
  return {{EQ, 0, 0, EQ, 1}, {EQ, 1, 1, EQ, 1}, {EQ, 0, 1, C, 1}, {EQ, 1, 0, B, 1},
          {C, 1, 0, C, 1},   {B, 0, 1, B, 1},   {Z, 0, 0, Z, 1},  {O, 1, 1, O, 1}};
}

std::vector<Step> accept_steps(const Factor& F) {
  const auto& f = F.f;
  std::vector<Step> all = {{EQ, 0, 0, 0, f[I_]},    {EQ, 1, 1, 0, f[I_]},   {EQ, 0, 1, 0, f[J_]},
                           {EQ, 1, 0, 0, f[JT_]},   {C, 1, 0, 0, f[J_]},    {B, 0, 1, 0, f[JT_]},
                           {Z, 0, 0, 0, f[E00_]},   {Z, 0, 1, 0, f[E01_]},  {Z, 1, 0, 0, f[E10_]},
                           {O, 1, 1, 0, f[ELL_]},   {O, 1, 0, 0, f[ELLM_]}, {O, 0, 1, 0, f[ELML_]}};
  std::vector<Step> out;
  for (const auto& s : all)
    if (s.v != 0.0) out.push_back(s);
  return out;
}

// Kronecker product over axes of per-axis step lists -> MPO nonzeros.
// state index: axis 0 most significant (radix nin[a] / nout[a] per axis); mode bits likewise.
void kron_steps(const std::vector<std::vector<Step>>& axes, const std::vector<int>& nin,
                const std::vector<int>& nout, MpoCore& core, int e_fixed) {
  const int D = (int)axes.size();
  std::vector<size_t> idx(D, 0);
  for (const auto& ax : axes)
    if (ax.empty()) return;
  while (true) {
    int s = 0, t = 0, io = 0, ii = 0;
    double v = 1.0;
    for (int a = 0; a < D; ++a) {
      const Step& st = axes[a][idx[a]];
      s = s * nin[a] + st.s;
      t = t * nout[a] + st.t;
      io = io * 2 + st.io;
      ii = ii * 2 + st.ii;
      v *= st.v;
    }
    if (v != 0.0) core.add(s, io, ii, e_fixed >= 0 ? e_fixed : t, v);
    int a = D - 1;
    while (a >= 0 && ++idx[a] == axes[a].size()) idx[a--] = 0;
    if (a < 0) break;
  }
}

// Young's modulus varying along one axis by one bit of the element index:
// element e (between nodes e and e + 1) has weight w[bit], bit = the level-L bit
// of e (levels most significant first).  The element-summed 1D factors of that
// axis then carry the weight on the steps of level L: the equal-prefix and J
// paths read it from the row bit, the J^T path from the column bit; the
// contribution of the element below a node (diagonal term d w(i - 1)) differs
// from w(i) only when the bits of i below level L are all zero, which the extra
// state LZ tracks with weight w(1 - bit) - w(bit).  The corner paths (Z, O) are
// not weighted; their coefficients are solved for the exact corner entries.
// The boundary atoms use the unweighted copy U of the equal-prefix path.
struct Layer {
  int axis = -1, L = 0;
  double w[2] = {1.0, 1.0};
};

std::vector<Step> level_steps(int l, const Layer* ly) {
  std::vector<Step> st = (l == 0) ? first_steps() : middle_steps();
  if (!ly) return st;
  const int src = (l == 0) ? 0 : EQ;
  if (l == ly->L) {
    for (auto& x : st) {
      if (x.t == EQ || x.t == C) x.v *= ly->w[x.io];
      else if (x.t == B) x.v *= ly->w[x.ii];
    }
    for (int b = 0; b < 2; ++b) st.push_back({src, b, b, LZ, ly->w[1 - b] - ly->w[b]});
  } else if (l > ly->L) {
    st.push_back({LZ, 0, 0, LZ, 1.0});
  }
  for (int b = 0; b < 2; ++b) st.push_back({l == 0 ? 0 : U, b, b, U, 1.0});
  return st;
}

std::vector<Step> accept_level_steps(const Factor& F, int d, const Layer* ly) {
  if (!ly) return accept_steps(F);
  const auto& f = F.f;
  std::vector<Step> all;
  if (ly->L < d - 1) {
    all = accept_steps(F);
    all.push_back({LZ, 0, 0, 0, f[LZ_]});
  } else {  // the weighted level is the last one
    const double* w = ly->w;
    all = {{EQ, 0, 0, 0, f[I_] * w[0] + f[LZ_] * (w[1] - w[0])},
           {EQ, 1, 1, 0, f[I_] * w[1] + f[LZ_] * (w[0] - w[1])},
           {EQ, 0, 1, 0, f[J_] * w[0]},
           {EQ, 1, 0, 0, f[JT_] * w[0]},
           {C, 1, 0, 0, f[J_] * w[1]},
           {B, 0, 1, 0, f[JT_] * w[1]},
           {Z, 0, 0, 0, f[E00_]},
           {Z, 0, 1, 0, f[E01_]},
           {Z, 1, 0, 0, f[E10_]},
           {O, 1, 1, 0, f[ELL_]},
           {O, 1, 0, 0, f[ELLM_]},
           {O, 0, 1, 0, f[ELML_]}};
  }
  all.push_back({U, 0, 0, 0, f[U_]});
  all.push_back({U, 1, 1, 0, f[U_]});
  std::vector<Step> out;
  for (const auto& x : all)
    if (x.v != 0.0) out.push_back(x);
  return out;
}

// Element-summed factor with element matrix [[a, b], [c, dd]] on a layered axis,
// masked at clamped ends (P F P): the coefficients of the weighted paths, and the
// corner coefficients that make the corner entries exact.
Factor layered_factor(double a, double b, double c, double dd, bool cl0, bool cl1, const Layer& ly, int d) {
  Factor F;
  F.f[I_] = a + dd;
  F.f[J_] = b;
  F.f[JT_] = c;
  F.f[LZ_] = dd;
  const double w0 = ly.w[0], w1 = ly.w[1];
  const double wN2 = ly.w[ly.L < d - 1 ? 1 : 0];  // weight of element N - 2
  // (0, 0): the low bits of node 0 are zero, so the LZ path reaches it
  F.f[E00_] = (cl0 ? 0.0 : a * w0) - ((a + dd) * w0 + dd * (w1 - w0));
  F.f[E01_] = cl0 ? -b * w0 : 0.0;
  F.f[E10_] = cl0 ? -c * w0 : 0.0;
  // (N-1, N-1): the bits of N - 1 below level L are all ones unless L is the last level
  const double pathLL = (a + dd) * w1 + (ly.L == d - 1 ? dd * (w0 - w1) : 0.0);
  F.f[ELL_] = (cl1 ? 0.0 : dd * wN2) - pathLL;
  F.f[ELLM_] = cl1 ? -c * wN2 : 0.0;
  F.f[ELML_] = cl1 ? -b * wN2 : 0.0;
  return F;
}

// Identity (and its masked form) on a layered axis: the unweighted path U, so the
// boundary atoms alpha (I - P) are the same as on a homogeneous axis.
Factor layered_identity(bool cl0, bool cl1) {
  Factor F;
  F.f[U_] = 1.0;
  if (cl0) F.f[E00_] = -1.0;
  if (cl1) F.f[ELL_] = -1.0;
  return F;
}

struct Atom {
  std::vector<Factor> axis;  // one factor per axis
  std::vector<double> comp;  // D x D component coefficients
};

// Dense TT-SVD of a vector of length 2^d into d QTT cores [r][2][r'].
}  // namespace

// QTT of a vector of 2^d entries by TT-SVD (relative accuracy 1e-15), levels most significant first.
std::vector<TTCore> vector_qtt(const std::vector<double>& v, int d) {
  std::vector<TTCore> cores;
  std::vector<double> rest = v;  // r x cols, row-major
  int r = 1;
  size_t cols = v.size();
  double nrm = 0;
  for (double x : v) nrm += x * x;
  nrm = std::sqrt(nrm);
  const double delta = 1e-15 * nrm / std::sqrt(std::max(d - 1, 1));
  for (int k = 0; k < d - 1; ++k) {
    const int m = r * 2;
    const size_t nc = cols / 2;
    // rest as m x nc matrix (row-major), SVD
    std::vector<double> U, S, Vt;
    hostla::svd(m, (int)nc, rest.data(), U, S, Vt);
    const int c = (int)S.size();
    // truncation: drop tail <= delta (absolute)
    double tail = 0;
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
    core.n = 2;
    core.rr = rk;
    core.data.resize((size_t)m * rk);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < rk; ++j) core.data[(size_t)i * rk + j] = U[(size_t)i * c + j];
    cores.push_back(core);
    std::vector<double> nr((size_t)rk * nc);
    for (int i = 0; i < rk; ++i)
      for (size_t j = 0; j < nc; ++j) nr[i * nc + j] = S[i] * Vt[(size_t)i * nc + j];
    rest.swap(nr);
    r = rk;
    cols = nc;
  }
  TTCore last;
  last.rl = r;
  last.n = 2;
  last.rr = 1;
  last.data = rest;
  cores.push_back(last);
  return cores;
}

// Level cores of a Kronecker product of per-axis QTT vectors (axis 0 most significant).
std::vector<TTCore> kron_vector_levels(const std::vector<std::vector<TTCore>>& axes) {
  const int d = (int)axes[0].size();
  std::vector<TTCore> out;
  for (int l = 0; l < d; ++l) {
    TTCore C = axes[0][l];
    for (size_t a = 1; a < axes.size(); ++a) {
      const TTCore& F = axes[a][l];
      TTCore N;
      N.rl = C.rl * F.rl;
      N.n = C.n * F.n;
      N.rr = C.rr * F.rr;
      N.data.assign((size_t)N.rl * N.n * N.rr, 0.0);
      for (int a1 = 0; a1 < C.rl; ++a1)
        for (int a2 = 0; a2 < F.rl; ++a2)
          for (int i1 = 0; i1 < C.n; ++i1)
            for (int i2 = 0; i2 < F.n; ++i2)
              for (int b1 = 0; b1 < C.rr; ++b1)
                for (int b2 = 0; b2 < F.rr; ++b2) {
                  const double x = C.data[((size_t)a1 * C.n + i1) * C.rr + b1] *
                                   F.data[((size_t)a2 * F.n + i2) * F.rr + b2];
                  N.data[(((size_t)(a1 * F.rl + a2)) * N.n + (i1 * F.n + i2)) * N.rr + (b1 * F.rr + b2)] = x;
                }
      C = N;
    }
    out.push_back(C);
  }
  return out;
}

// Direct sum of two TTs with equal modes (first core joined along the right bond,
// last core along the left bond, middle cores block diagonal).
std::vector<TTCore> tt_sum(const std::vector<TTCore>& x, const std::vector<TTCore>& y) {
  const size_t K = x.size();
  std::vector<TTCore> out(K);
  for (size_t k = 0; k < K; ++k) {
    const TTCore &a = x[k], &b = y[k];
    TTCore c;
    c.n = a.n;
    c.rl = (k == 0) ? 1 : a.rl + b.rl;
    c.rr = (k == K - 1) ? 1 : a.rr + b.rr;
    c.data.assign((size_t)c.rl * c.n * c.rr, 0.0);
    const int ol = (k == 0) ? 0 : a.rl, orr = (k == K - 1) ? 0 : a.rr;
    for (int i = 0; i < a.rl; ++i)
      for (int j = 0; j < a.n; ++j)
        for (int l = 0; l < a.rr; ++l) c.data[((size_t)i * c.n + j) * c.rr + l] = a.data[((size_t)i * a.n + j) * a.rr + l];
    for (int i = 0; i < b.rl; ++i)
      for (int j = 0; j < b.n; ++j)
        for (int l = 0; l < b.rr; ++l)
          c.data[((size_t)(i + ol) * c.n + j) * c.rr + (l + orr)] += b.data[((size_t)i * b.n + j) * b.rr + l];
    out[k] = c;
  }
  return out;
}

namespace {

// ----------------------------------------------------------------------------- nodal load f0

// A 1D operator in QTT form: d cores [R][2][2][R'] (output bit, input bit), most
// significant level first, boundary ranks 1.
struct Qtt1d {
  std::vector<int> r;                    // d + 1 ranks
  std::vector<std::vector<double>> c;    // d cores
  double coef = 1.0;
};

// Per-level 2 x 2 blocks (output bit, input bit).
static const double I2[4] = {1, 0, 0, 1};
static const double J2[4] = {0, 1, 0, 0};   // (0, 1): the input index is the output index + 1
static const double J2t[4] = {0, 0, 1, 0};  // (1, 0)
static const double E0[4] = {1, 0, 0, 0};
static const double E1[4] = {0, 0, 0, 1};

// Rank-1 Kronecker product of per-level blocks: blk(l) for l < d - 1, last for l = d - 1.
static Qtt1d qtt1d_rank1(int d, const double* blk, const double* last, double coef) {
  Qtt1d q;
  q.coef = coef;
  q.r.assign(d + 1, 1);
  for (int l = 0; l < d; ++l) q.c.emplace_back(l == d - 1 ? last : blk, (l == d - 1 ? last : blk) + 4);
  return q;
}

// The upper shift J (J[i][j] = 1 iff j = i + 1), or its transpose: a carry automaton
// whose bond state is the carry passed from the less significant levels (right bond:
// carry into the level, left bond: carry out of it).  Without a carry the bits agree;
// with one the level either absorbs it (bits 0 -> 1 for J) or passes it on (1 -> 0).
static Qtt1d qtt1d_shift(int d, bool transpose, double coef) {
  const double* up = transpose ? J2t : J2;    // carry absorbed
  const double* pass = transpose ? J2 : J2t;  // carry passed on
  Qtt1d q;
  q.coef = coef;
  q.r.assign(d + 1, 2);
  q.r[0] = 1;
  q.r[d] = 1;
  for (int l = 0; l < d; ++l) {
    const int rl = q.r[l], rr = q.r[l + 1];
    std::vector<double> c((size_t)rl * 4 * rr, 0.0);
    auto put = [&](int a, int b, const double* m) {
      for (int e = 0; e < 4; ++e) c[((size_t)a * 4 + e) * rr + b] = m[e];
    };
    if (d == 1) {
      put(0, 0, up);  // one level: the carry enters and must be absorbed
    } else if (l == 0) {
      put(0, 0, I2);  // no overflow out of the most significant level
      put(0, 1, up);
    } else if (l == d - 1) {
      put(0, 0, up);  // the +1 enters at the least significant level
      put(1, 0, pass);
    } else {
      put(0, 0, I2);
      put(0, 1, up);
      put(1, 1, pass);
    }
    q.c.push_back(c);
  }
  return q;
}

// Terms of P_a M_a, the 1D consistent mass matrix of axis a with the rows of clamped
// ends removed:  M = h/6 (4 I + J + J^T - 2 E00 - 2 Ell),  E00 M = h/6 (2 E00 + E00 J),
// Ell M = h/6 (2 Ell + Ell J^T),  P_a M = M - c0 E00 M - c1 Ell M.
static std::vector<Qtt1d> masked_mass_terms(int d, double h, bool c0, bool c1) {
  const double s = h / 6.0;
  std::vector<Qtt1d> t;
  t.push_back(qtt1d_rank1(d, I2, I2, 4 * s));
  t.push_back(qtt1d_shift(d, false, s));
  t.push_back(qtt1d_shift(d, true, s));
  t.push_back(qtt1d_rank1(d, E0, E0, -(2.0 + 2.0 * c0) * s));
  t.push_back(qtt1d_rank1(d, E1, E1, -(2.0 + 2.0 * c1) * s));
  if (c0) t.push_back(qtt1d_rank1(d, E0, J2, -s));   // e_0 e_1^T
  if (c1) t.push_back(qtt1d_rank1(d, E1, J2t, -s));  // e_l e_{l-1}^T
  return t;
}

// Applies the 1D operator op to the bits of axis a of a TT in the solution layout (d level
// cores of mode 2^D, mode bit of axis a at position D - 1 - a, then the component core).
static std::vector<TTCore> apply_axis(const std::vector<TTCore>& X, const Qtt1d& op, int a, int D) {
  const int d = (int)X.size() - 1;
  const int nm = 1 << D, shift = D - 1 - a;
  std::vector<TTCore> Y(d + 1);
  for (int l = 0; l < d; ++l) {
    const TTCore& x = X[l];
    const int Rl = op.r[l], Rr = op.r[l + 1];
    TTCore y;
    y.rl = x.rl * Rl;
    y.n = nm;
    y.rr = x.rr * Rr;
    y.data.assign((size_t)y.rl * nm * y.rr, 0.0);
    const std::vector<double>& c = op.c[l];
    for (int al = 0; al < x.rl; ++al)
      for (int mo = 0; mo < nm; ++mo) {
        const int bo = (mo >> shift) & 1;
        for (int bi = 0; bi < 2; ++bi) {
          const int mi = (mo & ~(1 << shift)) | (bi << shift);
          for (int rho = 0; rho < Rl; ++rho)
            for (int sg = 0; sg < Rr; ++sg) {
              const double w = c[((size_t)rho * 4 + bo * 2 + bi) * Rr + sg];
              if (w == 0.0) continue;
              for (int be = 0; be < x.rr; ++be)
                y.data[(((size_t)al * Rl + rho) * nm + mo) * y.rr + (size_t)be * Rr + sg] +=
                    w * x.data[((size_t)al * nm + mi) * x.rr + be];
            }
        }
      }
    Y[l] = y;
  }
  Y[d] = X[d];
  for (double& v : Y[0].data) v *= op.coef;
  return Y;
}

}  // namespace

size_t f0_doubles(const tnfem_problem_desc& desc) {
  if (!desc.f0_cores) return 0;
  TNFEM_REQUIRE(desc.f0_ranks != nullptr, "f0_cores given without f0_ranks");
  const int D = desc.dim, d = desc.level;
  TNFEM_REQUIRE((D == 2 || D == 3) && d >= 2 && d <= 20, "invalid dim or level");
  const int K = d + 1;
  TNFEM_REQUIRE(desc.f0_ranks[0] == 1 && desc.f0_ranks[K] == 1, "f0 boundary ranks must be 1");
  size_t total = 0;
  for (int k = 0; k < K; ++k) {
    const int rl = desc.f0_ranks[k], rr = desc.f0_ranks[k + 1];
    TNFEM_REQUIRE(rl >= 1 && rl <= 4096 && rr >= 1 && rr <= 4096, "f0 ranks must be in [1, 4096]");
    total += (size_t)rl * (k < d ? (1u << D) : (unsigned)D) * rr;
  }
  return total;
}

// P M f0 in TT format: one axis at a time, the masked 1D mass terms applied, summed and
// rounded.
static std::vector<TTCore> nodal_load(const tnfem_problem_desc& desc, const bool* c0, const bool* c1) {
  const int D = desc.dim, d = desc.level, K = d + 1;
  f0_doubles(desc);  // validates
  std::vector<TTCore> X(K);
  size_t off = 0;
  for (int k = 0; k < K; ++k) {
    X[k].rl = desc.f0_ranks[k];
    X[k].rr = desc.f0_ranks[k + 1];
    X[k].n = k < d ? (1 << D) : D;
    const size_t sz = (size_t)X[k].rl * X[k].n * X[k].rr;
    X[k].data.assign(desc.f0_cores + off, desc.f0_cores + off + sz);
    for (double v : X[k].data) TNFEM_REQUIRE(std::isfinite(v), "f0 holds a non-finite value");
    off += sz;
  }
  const int n = 1 << d;
  for (int a = 0; a < D; ++a) {
    const double h = desc.extent[a] / (n - 1);
    std::vector<TTCore> acc;
    for (const Qtt1d& op : masked_mass_terms(d, h, c0[a], c1[a])) {
      std::vector<TTCore> y = apply_axis(X, op, a, D);
      acc = acc.empty() ? y : tt_sum(acc, y);
    }
    tt_round_host(acc, 1e-14, 1 << 30);
    X = acc;
  }
  return X;
}

void tt_round_host(std::vector<TTCore>& cores, double tol, int rmax) {
  const int K = (int)cores.size();
  if (K == 1) return;
  // right-to-left orthogonalisation: core k = L Q with Q row-orthonormal
  for (int k = K - 1; k > 0; --k) {
    TTCore& c = cores[k];
    const int rows = c.rl, cols = c.n * c.rr;
    std::vector<double> T((size_t)cols * rows);
    for (int i = 0; i < rows; ++i)
      for (int j = 0; j < cols; ++j) T[(size_t)j * rows + i] = c.data[(size_t)i * cols + j];
    std::vector<double> Q, R;
    hostla::qr(cols, rows, T.data(), Q, R);  // Q cols x q, R q x rows
    const int q = std::min(cols, rows);
    TTCore nc;
    nc.rl = q;
    nc.n = c.n;
    nc.rr = c.rr;
    nc.data.resize((size_t)q * cols);
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < cols; ++j) nc.data[(size_t)i * cols + j] = Q[(size_t)j * q + i];
    // previous core times R^T
    TTCore& p = cores[k - 1];
    const int pr = p.rl * p.n;
    std::vector<double> np((size_t)pr * q, 0.0);
    for (int i = 0; i < pr; ++i)
      for (int a = 0; a < rows; ++a) {
        const double x = p.data[(size_t)i * rows + a];
        if (x == 0.0) continue;
        for (int j = 0; j < q; ++j) np[(size_t)i * q + j] += x * R[(size_t)j * rows + a];
      }
    p.rr = q;
    p.data.swap(np);
    c = nc;
  }
  double nrm = 0;
  for (double x : cores[0].data) nrm += x * x;
  nrm = std::sqrt(nrm);
  const double delta_rel = tol / std::sqrt((double)std::max(K - 1, 1));
  for (int k = 0; k < K - 1; ++k) {
    TTCore& c = cores[k];
    const int m = c.rl * c.n, n = c.rr;
    std::vector<double> U, S, Vt;
    hostla::svd(m, n, c.data.data(), U, S, Vt);
    const int cc = (int)S.size();
    // absolute threshold relative to the whole TT norm
    double tail = 0;
    int rk = cc;
    for (int j = cc - 1; j >= 1; --j) {
      if (tail + S[j] * S[j] <= delta_rel * delta_rel * nrm * nrm) {
        tail += S[j] * S[j];
        rk = j;
      } else {
        break;
      }
    }
    rk = std::max(1, std::min(rk, rmax));
    TTCore nc;
    nc.rl = c.rl;
    nc.n = c.n;
    nc.rr = rk;
    nc.data.resize((size_t)m * rk);
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < rk; ++j) nc.data[(size_t)i * rk + j] = U[(size_t)i * cc + j];
    TTCore& nx = cores[k + 1];
    const int cols = nx.n * nx.rr;
    std::vector<double> W((size_t)rk * n);
    for (int i = 0; i < rk; ++i)
      for (int j = 0; j < n; ++j) W[(size_t)i * n + j] = S[i] * Vt[(size_t)i * n + j];
    std::vector<double> nd((size_t)rk * cols, 0.0);
    hostla::gemm(rk, cols, n, W.data(), nx.data.data(), nd.data());
    nx.rl = rk;
    nx.data.swap(nd);
    c = nc;
  }
}

// Index of the Voigt component of the symmetric pair (i, j): 2D (xx, yy, xy), 3D (xx, yy, zz,
// yz, xz, xy).
static int voigt(int D, int i, int j) {
  if (i == j) return i;
  if (D == 2) return 2;
  return i + j == 3 ? 3 : (i + j == 2 ? 4 : 5);  // yz, xz, xy
}

std::vector<double> stiffness_tensor(const tnfem_problem_desc& desc, int D, double lam, double mu) {
  std::vector<double> C((size_t)D * D * D * D, 0.0);
  auto at = [&](int i, int a, int j, int b) -> double& { return C[((i * D + a) * D + j) * D + b]; };
  if (!desc.has_stiffness) {
    for (int i = 0; i < D; ++i)
      for (int a = 0; a < D; ++a)
        for (int j = 0; j < D; ++j)
          for (int b = 0; b < D; ++b)
            at(i, a, j, b) = lam * (i == a) * (j == b) + mu * ((i == j) * (a == b) + (i == b) * (a == j));
    return C;
  }
  const int nv = D == 2 ? 3 : 6;
  std::vector<double> V((size_t)nv * nv);
  for (int r = 0; r < nv; ++r)
    for (int c = 0; c < nv; ++c) {
      V[(size_t)r * nv + c] = desc.stiffness[r][c];
      TNFEM_REQUIRE(std::isfinite(desc.stiffness[r][c]), "stiffness holds a non-finite value");
    }
  double scale = 0.0;
  for (double v : V) scale = std::max(scale, std::fabs(v));
  for (int r = 0; r < nv; ++r)
    for (int c = 0; c < r; ++c)
      TNFEM_REQUIRE(std::fabs(V[(size_t)r * nv + c] - V[(size_t)c * nv + r]) <= 1e-12 * scale,
                    "stiffness must be symmetric");
  // positive definite: Cholesky
  std::vector<double> L = V;
  for (int j = 0; j < nv; ++j) {
    double dj = L[(size_t)j * nv + j];
    for (int k = 0; k < j; ++k) dj -= L[(size_t)j * nv + k] * L[(size_t)j * nv + k];
    TNFEM_REQUIRE(dj > 1e-14 * scale, "stiffness must be positive definite");
    dj = std::sqrt(dj);
    L[(size_t)j * nv + j] = dj;
    for (int i = j + 1; i < nv; ++i) {
      double v = L[(size_t)i * nv + j];
      for (int k = 0; k < j; ++k) v -= L[(size_t)i * nv + k] * L[(size_t)j * nv + k];
      L[(size_t)i * nv + j] = v / dj;
    }
  }
  for (int i = 0; i < D; ++i)
    for (int a = 0; a < D; ++a)
      for (int j = 0; j < D; ++j)
        for (int b = 0; b < D; ++b) at(i, a, j, b) = V[(size_t)voigt(D, i, a) * nv + voigt(D, j, b)];
  return C;
}

Assembled assemble(const tnfem_problem_desc& desc) {
  if (desc.has_quad) return assemble_quad(desc);
  if (desc.elem_weight) {
    // a per-element field on a 2D box: the quadrilateral path on the rectangle
    TNFEM_REQUIRE(desc.dim == 2, "elem_weight is a 2D option");
    tnfem_problem_desc q = desc;
    q.has_quad = 1;
    const double c[4][2] = {{0.0, 0.0}, {desc.extent[0], 0.0}, {0.0, desc.extent[1]}, {desc.extent[0], desc.extent[1]}};
    for (int i = 0; i < 4; ++i)
      for (int k = 0; k < 2; ++k) q.quad[i][k] = c[i][k];
    return assemble_quad(q);
  }
  const int D = desc.dim, d = desc.level;
  TNFEM_REQUIRE(D == 2 || D == 3, "dim must be 2 or 3 (got %d)", D);
  TNFEM_REQUIRE(d >= 2 && d <= 20, "level must be in [2, 20] (got %d)", d);
  TNFEM_REQUIRE(desc.E > 0 && std::isfinite(desc.E), "E must be positive");
  TNFEM_REQUIRE(desc.nu > -1.0 && desc.nu < 0.5, "nu must be in (-1, 0.5)");
  for (int a = 0; a < D; ++a) TNFEM_REQUIRE(desc.extent[a] > 0, "extent[%d] must be positive", a);
  TNFEM_REQUIRE(!(desc.plane_stress && D == 3), "plane_stress is a 2D option");
  TNFEM_REQUIRE(!(desc.plane_stress && desc.has_stiffness), "plane_stress does not combine with a stiffness matrix");
  TNFEM_REQUIRE(!(desc.has_manufactured && desc.has_stiffness),
                "the manufactured load is the isotropic closed form; it does not combine with a stiffness matrix");
  TNFEM_REQUIRE((desc.clamp_mask >> (2 * D)) == 0, "clamp_mask names a face beyond dim");
  TNFEM_REQUIRE(desc.n_tractions >= 0 && desc.n_tractions <= 6, "n_tractions must be in [0, 6]");
  const int n = 1 << d;
  Layer ly;
  const bool layered = desc.layer_E != nullptr;
  if (layered) {
    TNFEM_REQUIRE(desc.layer_axis >= 0 && desc.layer_axis < D, "layer_axis must be in [0, dim)");
    TNFEM_REQUIRE(desc.n_layer_E == n - 1, "layer_E must hold one value per element layer (%d)", n - 1);
    std::vector<double> w(n - 1);
    for (int e = 0; e < n - 1; ++e) {
      w[e] = desc.layer_E[e] / desc.E;
      TNFEM_REQUIRE(w[e] > 0 && std::isfinite(w[e]), "layer_E must be positive");
    }
    bool found = false;
    for (int L = 0; L < d && !found; ++L) {
      double v[2] = {NAN, NAN};
      bool ok = true;
      for (int e = 0; e < n - 1 && ok; ++e) {
        const int bit = (e >> (d - 1 - L)) & 1;
        if (std::isnan(v[bit])) v[bit] = w[e];
        else ok = v[bit] == w[e];
      }
      if (ok) {
        found = true;
        ly.axis = desc.layer_axis;
        ly.L = L;
        ly.w[0] = v[0];
        ly.w[1] = v[1];
      }
    }
    TNFEM_REQUIRE(found,
                  "layer_E must be a function of one bit of the element index along layer_axis "
                  "(slabs alternating every 2^k element layers)");
  }

  Assembled out;
  out.D = D;
  out.d = d;
  double lam = desc.E * desc.nu / ((1 + desc.nu) * (1 - 2 * desc.nu));
  double mu = desc.E / (2 * (1 + desc.nu));
  if (desc.plane_stress) lam = 2 * lam * mu / (lam + 2 * mu);
  // stiffness tensor C[i][a][j][b]: sigma_ia = sum_jb C_iajb du_j/dx_b
  std::vector<double> Ct = stiffness_tensor(desc, D, lam, mu);
  auto Cq = [&](int i, int a, int j, int b) { return Ct[((i * D + a) * D + j) * D + b]; };
  double cmax = 0.0;
  for (int i = 0; i < D; ++i) cmax = std::max(cmax, Cq(i, i, i, i));
  const double h0 = desc.extent[0] / (n - 1);
  const double alpha = cmax * std::pow(h0, D - 2);
  out.lam = lam;
  out.mu = mu;
  out.alpha = alpha;

  bool c0[3] = {false, false, false}, c1[3] = {false, false, false};
  bool any_clamp = false;
  for (int a = 0; a < D; ++a) {
    c0[a] = (desc.clamp_mask >> (2 * a)) & 1;
    c1[a] = (desc.clamp_mask >> (2 * a + 1)) & 1;
    any_clamp = any_clamp || c0[a] || c1[a];
  }

  // 1D factors per axis (closed forms of the element integrals, summed over elements)
  std::vector<Factor> S(D), M(D), G(D), GT(D), Id(D), P(D);
  for (int a = 0; a < D; ++a) {
    const double h = desc.extent[a] / (n - 1);
    Factor s, m, g, gt, id;
    s.f[I_] = 2 / h; s.f[J_] = -1 / h; s.f[JT_] = -1 / h; s.f[E00_] = -1 / h; s.f[ELL_] = -1 / h;
    m.f[I_] = 4 * h / 6; m.f[J_] = h / 6; m.f[JT_] = h / 6; m.f[E00_] = -2 * h / 6; m.f[ELL_] = -2 * h / 6;
    g.f[J_] = -0.5; g.f[JT_] = 0.5; g.f[E00_] = -0.5; g.f[ELL_] = 0.5;
    gt.f[J_] = 0.5; gt.f[JT_] = -0.5; gt.f[E00_] = -0.5; gt.f[ELL_] = 0.5;
    id.f[I_] = 1;
    S[a] = masked(s, c0[a], c1[a]);
    M[a] = masked(m, c0[a], c1[a]);
    G[a] = masked(g, c0[a], c1[a]);
    GT[a] = masked(gt, c0[a], c1[a]);
    Id[a] = id;
    P[a] = masked(id, c0[a], c1[a]);
    if (layered && a == ly.axis) {  // element matrices [[a, b], [c, d]] of S, M, G, G^T
      S[a] = layered_factor(1 / h, -1 / h, -1 / h, 1 / h, c0[a], c1[a], ly, d);
      M[a] = layered_factor(2 * h / 6, h / 6, h / 6, 2 * h / 6, c0[a], c1[a], ly, d);
      G[a] = layered_factor(-0.5, -0.5, 0.5, 0.5, c0[a], c1[a], ly, d);
      GT[a] = layered_factor(-0.5, 0.5, -0.5, 0.5, c0[a], c1[a], ly, d);
      Id[a] = layered_identity(false, false);
      P[a] = layered_identity(c0[a], c1[a]);
    }
  }

  std::vector<Atom> atoms;
  for (int a = 0; a < D; ++a)
    for (int b = 0; b < D; ++b) {
      Atom at;
      for (int c = 0; c < D; ++c) {
        if (a == b) at.axis.push_back(c == a ? S[c] : M[c]);
        else at.axis.push_back(c == a ? G[c] : (c == b ? GT[c] : M[c]));
      }
      // test component i, trial component j of the term d_a phi_p d_b phi_q
      at.comp.assign(D * D, 0.0);
      for (int i = 0; i < D; ++i)
        for (int j = 0; j < D; ++j) at.comp[i * D + j] = Cq(i, a, j, b);
      atoms.push_back(at);
    }
  if (any_clamp) {
    Atom ia, pa;
    ia.axis = Id;
    pa.axis = P;
    ia.comp.assign(D * D, 0.0);
    pa.comp.assign(D * D, 0.0);
    for (int c = 0; c < D; ++c) {
      ia.comp[c * D + c] = alpha;
      pa.comp[c * D + c] = -alpha;
    }
    atoms.push_back(ia);
    atoms.push_back(pa);
  }
  const int nat = (int)atoms.size();
  std::vector<int> nsa(D, NSTATE);  // automaton states per axis
  if (layered) nsa[ly.axis] = NSTATE + 2;
  int ns = 1;
  for (int a = 0; a < D; ++a) ns *= nsa[a];
  const int nm = 1 << D;
  auto layer_of = [&](int a) { return (layered && a == ly.axis) ? &ly : nullptr; };

  // level cores
  for (int l = 0; l < d; ++l) {
    MpoCore core;
    core.n = nm;
    if (l < d - 1) {
      core.Rl = l == 0 ? 1 : ns;
      core.Rr = ns;
      std::vector<std::vector<Step>> axes;
      std::vector<int> rin, rout;
      for (int a = 0; a < D; ++a) {
        axes.push_back(level_steps(l, layer_of(a)));
        rin.push_back(l == 0 ? 1 : nsa[a]);
        rout.push_back(nsa[a]);
      }
      kron_steps(axes, rin, rout, core, -1);
    } else {
      core.Rl = ns;
      core.Rr = nat;
      for (int t = 0; t < nat; ++t) {
        std::vector<std::vector<Step>> axes;
        for (int a = 0; a < D; ++a) axes.push_back(accept_level_steps(atoms[t].axis[a], d, layer_of(a)));
        kron_steps(axes, nsa, std::vector<int>(D, 1), core, t);
      }
    }
    out.A.push_back(core);
  }
  // component core [nat][D][D][1]
  {
    MpoCore core;
    core.Rl = nat;
    core.Rr = 1;
    core.n = D;
    for (int t = 0; t < nat; ++t)
      for (int a = 0; a < D; ++a)
        for (int b = 0; b < D; ++b)
          if (atoms[t].comp[a * D + b] != 0.0) core.add(t, a, b, 0, atoms[t].comp[a * D + b]);
    out.A.push_back(core);
  }

  // ---- load: sum of (component vector) x (Kronecker product of 1D nodal vectors)
  struct LoadTerm {
    std::vector<double> comp;
    std::vector<std::vector<double>> vec;
  };
  std::vector<LoadTerm> terms;
  auto mass_times = [&](int a, const std::vector<double>& v) {
    const double h = desc.extent[a] / (n - 1);
    std::vector<double> r(n);
    for (int i = 0; i < n; ++i) {
      const double left = i > 0 ? v[i - 1] : 0.0, right = i < n - 1 ? v[i + 1] : 0.0;
      const double diag = (i == 0 || i == n - 1) ? 2.0 : 4.0;
      r[i] = h / 6.0 * (left + diag * v[i] + right);
    }
    return r;
  };
  auto mask_vec = [&](int a, std::vector<double> v) {
    if (c0[a]) v[0] = 0.0;
    if (c1[a]) v[n - 1] = 0.0;
    return v;
  };
  const std::vector<double> ones(n, 1.0);
  if (desc.has_body_force) {
    LoadTerm t;
    t.comp.assign(desc.body_force, desc.body_force + D);
    for (int a = 0; a < D; ++a) t.vec.push_back(mask_vec(a, mass_times(a, ones)));
    terms.push_back(t);
  }
  for (int q = 0; q < desc.n_tractions; ++q) {
    const int face = desc.traction_face[q];
    TNFEM_REQUIRE(face >= 0 && face < 2 * D, "traction face %d out of range", face);
    const int ax = face / 2, side = face % 2;
    LoadTerm t;
    t.comp.assign(desc.traction[q], desc.traction[q] + D);
    for (int a = 0; a < D; ++a) {
      if (a == ax) {
        std::vector<double> e(n, 0.0);
        e[side ? n - 1 : 0] = 1.0;
        t.vec.push_back(mask_vec(a, e));
      } else {
        t.vec.push_back(mask_vec(a, mass_times(a, ones)));
      }
    }
    terms.push_back(t);
  }
  if (desc.has_manufactured) {
    const double* c = desc.manufactured_c;
    const double pi = 3.14159265358979323846;
    std::vector<std::vector<double>> sv(D), kv(D);
    for (int a = 0; a < D; ++a) {
      std::vector<double> s(n), k(n);
      for (int i = 0; i < n; ++i) {
        const double x = i * desc.extent[a] / (n - 1);
        s[i] = std::sin(pi * x);
        k[i] = std::cos(pi * x);
      }
      sv[a] = mask_vec(a, mass_times(a, s));
      kv[a] = mask_vec(a, mass_times(a, k));
    }
    // -div sigma(u*) with u*_i = c_i prod sin(pi x_a): separable terms
    for (int i = 0; i < D; ++i) {
      LoadTerm t;
      t.comp.assign(D, 0.0);
      t.comp[i] = pi * pi * (lam + (D + 1) * mu) * c[i];
      for (int a = 0; a < D; ++a) t.vec.push_back(sv[a]);
      terms.push_back(t);
      for (int k = 0; k < D; ++k) {
        if (k == i) continue;
        LoadTerm u;
        u.comp.assign(D, 0.0);
        u.comp[i] = -pi * pi * (lam + mu) * c[k];
        for (int a = 0; a < D; ++a) u.vec.push_back((a == i || a == k) ? kv[a] : sv[a]);
        terms.push_back(u);
      }
    }
  }
  std::vector<TTCore> total;
  for (const auto& t : terms) {
    std::vector<std::vector<TTCore>> axes;
    for (int a = 0; a < D; ++a) axes.push_back(vector_qtt(t.vec[a], d));
    std::vector<TTCore> lev = kron_vector_levels(axes);
    TTCore cc;
    cc.rl = 1;
    cc.n = D;
    cc.rr = 1;
    cc.data = t.comp;
    lev.push_back(cc);
    if (total.empty()) {
      total = lev;
    } else {
      total = tt_sum(total, lev);
      tt_round_host(total, 1e-14, 1 << 30);
    }
  }
  if (desc.f0_cores) {
    std::vector<TTCore> f0b = nodal_load(desc, c0, c1);
    if (total.empty()) {
      total = f0b;
    } else {
      total = tt_sum(total, f0b);
      tt_round_host(total, 1e-14, 1 << 30);
    }
  }
  if (total.empty()) {
    for (int l = 0; l < d; ++l) {
      TTCore z;
      z.n = nm;
      z.data.assign(nm, 0.0);
      total.push_back(z);
    }
    TTCore z;
    z.n = D;
    z.data.assign(D, 0.0);
    total.push_back(z);
  }
  out.b = total;
  return out;
}

}  // namespace tnfem
