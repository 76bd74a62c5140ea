// Host assembly of the QTT operator and load (Alg. 1 on the Cartesian grid).
#pragma once

#include <vector>

#include "../../include/tnfem.h"

namespace tnfem {

// One MPO core as a list of nonzeros A[b][io][ii][e] = v (io: output mode, ii: input mode).
struct MpoCore {
  int Rl = 1, Rr = 1, n = 1;
  std::vector<int> b, io, ii, e;
  std::vector<double> v;
  void add(int b_, int io_, int ii_, int e_, double v_) {
    b.push_back(b_); io.push_back(io_); ii.push_back(ii_); e.push_back(e_); v.push_back(v_);
  }
  size_t nnz() const { return v.size(); }
  std::vector<double> dense() const;  // [Rl][n][n][Rr]
};

// One TT core, row-major [rl][n][rr].
struct TTCore {
  int rl = 1, n = 1, rr = 1;
  std::vector<double> data;
};

struct Assembled {
  int D = 2, d = 2;
  double lam = 0, mu = 0, alpha = 0;
  std::vector<MpoCore> A;  // d level cores, then the component core
  std::vector<TTCore> b;   // load, same layout
};

// Validates desc (throws tnfem::Error) and assembles operator and load.
Assembled assemble(const tnfem_problem_desc& desc);

// Stiffness tensor C[((i D + a) D + j) D + b] (sigma_ia = sum C_iajb du_j/dx_b): the desc's Voigt
// matrix when has_stiffness (validated: symmetric positive definite), else the isotropic law.
std::vector<double> stiffness_tensor(const tnfem_problem_desc& desc, int D, double lam, double mu);

// Doubles of the nodal load f0 (0 without one); validates its ranks (throws tnfem::Error).
size_t f0_doubles(const tnfem_problem_desc& desc);

// QTT of a vector of 2^d entries (levels most significant first) by TT-SVD.
std::vector<TTCore> vector_qtt(const std::vector<double>& v, int d);
// Level cores of the Kronecker product of per-axis QTT vectors (axis 0 most significant bit).
std::vector<TTCore> kron_vector_levels(const std::vector<std::vector<TTCore>>& axes);
// Direct sum of two TTs with equal modes (ranks add).
std::vector<TTCore> tt_sum(const std::vector<TTCore>& x, const std::vector<TTCore>& y);

// Operator and load on a quadrilateral domain (desc.has_quad; 2D), Alg. 1 with the element
// Jacobians frozen at the element centres.
Assembled assemble_quad(const tnfem_problem_desc& desc);

// TT rounding on the host (relative accuracy tol, at most rmax).
void tt_round_host(std::vector<TTCore>& cores, double tol, int rmax);

}  // namespace tnfem
