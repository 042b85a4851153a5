// Scalar types for the serial reference solver ("oracle").
//
// TEST INFRASTRUCTURE ONLY. This directory is the CPU oracle that the HIP
// path is checked against; only the test suite, the smoke check and the
// CPU-baseline leg of the benchmark load it. Product code never includes,
// links or calls anything here.
//
// The solver in cfd_oracle.cpp is written once, templated on its scalar, and
// instantiated three times:
//   double   - the forward solver;
//   OpCount  - a double that counts every arithmetic operation it performs,
//              which gives the algorithmic operation count per cell update;
//   TVar     - a minimal reverse-mode automatic-differentiation variable that
//              records a tape. Reversing the tape gives the exact derivative of
//              the oracle's own discrete operator, independently of any
//              hand-derived adjoint formula.
// Every branch of the solver decides on val(x), so all three instantiations
// follow exactly the same control flow.
#pragma once
#include <cmath>
#include <cstdint>
#include <vector>

namespace oracle {

// ---------------------------------------------------------------- double ---
inline double val(double x) { return x; }
inline double sqrt_(double x) { return std::sqrt(x); }
inline double abs_(double x) { return std::fabs(x); }
// Ties pick the first argument; the adjoint follows the same rule.
inline double min_(double a, double b) { return (b < a) ? b : a; }
inline double max_(double a, double b) { return (b > a) ? b : a; }
inline double exp_(double x) { return std::exp(x); }
inline double log_(double x) { return std::log(x); }

// --------------------------------------------------------------- OpCount ---
struct OpTally {
  double add = 0, mul = 0, div = 0, sqrt = 0, cmp = 0;
};
inline OpTally& tally() {
  static thread_local OpTally t;
  return t;
}

struct OpCount {
  double v = 0.0;
  OpCount() = default;
  OpCount(double x) : v(x) {}  // NOLINT: implicit from constants
};
inline double val(const OpCount& x) { return x.v; }
inline OpCount operator+(OpCount a, OpCount b) { tally().add += 1; return OpCount(a.v + b.v); }
inline OpCount operator-(OpCount a, OpCount b) { tally().add += 1; return OpCount(a.v - b.v); }
inline OpCount operator*(OpCount a, OpCount b) { tally().mul += 1; return OpCount(a.v * b.v); }
inline OpCount operator/(OpCount a, OpCount b) { tally().div += 1; return OpCount(a.v / b.v); }
inline OpCount operator-(OpCount a) { return OpCount(-a.v); }
inline OpCount& operator+=(OpCount& a, OpCount b) { a = a + b; return a; }
inline OpCount& operator-=(OpCount& a, OpCount b) { a = a - b; return a; }
inline OpCount sqrt_(OpCount x) { tally().sqrt += 1; return OpCount(std::sqrt(x.v)); }
inline OpCount abs_(OpCount x) { tally().cmp += 1; return OpCount(std::fabs(x.v)); }
inline OpCount min_(OpCount a, OpCount b) { tally().cmp += 1; return (b.v < a.v) ? b : a; }
inline OpCount max_(OpCount a, OpCount b) { tally().cmp += 1; return (b.v > a.v) ? b : a; }
inline OpCount exp_(OpCount x) { tally().div += 1; return OpCount(std::exp(x.v)); }
inline OpCount log_(OpCount x) { tally().div += 1; return OpCount(std::log(x.v)); }

// ------------------------------------------------------------------ TVar ---
// Tape entry: the value y of an operation with at most two operands x1, x2
// and the local partial derivatives dy/dx1, dy/dx2. Operands with index < 0
// are constants.
struct TapeNode {
  int32_t a, b;
  double ga, gb;
};
struct Tape {
  std::vector<TapeNode> nodes;
  int32_t push(int32_t a, double ga, int32_t b, double gb) {
    nodes.push_back(TapeNode{a, b, ga, gb});
    return static_cast<int32_t>(nodes.size() - 1);
  }
  int32_t leaf() { return push(-1, 0.0, -1, 0.0); }
  // Reverse sweep: adj has one entry per node, seeded by the caller.
  void reverse(std::vector<double>& adj) const {
    for (int64_t i = static_cast<int64_t>(nodes.size()) - 1; i >= 0; --i) {
      const double g = adj[i];
      if (g == 0.0) continue;
      const TapeNode& n = nodes[i];
      if (n.a >= 0) adj[n.a] += g * n.ga;
      if (n.b >= 0) adj[n.b] += g * n.gb;
    }
  }
};
inline Tape*& active_tape() {
  static thread_local Tape* t = nullptr;
  return t;
}

struct TVar {
  double v = 0.0;
  int32_t id = -1;  // -1: constant, not on the tape
  TVar() = default;
  TVar(double x) : v(x), id(-1) {}  // NOLINT: implicit from constants
  static TVar make(double v, int32_t a, double ga, int32_t b, double gb) {
    TVar r(v);
    if (a >= 0 || b >= 0) r.id = active_tape()->push(a, ga, b, gb);
    return r;
  }
  static TVar leaf(double v) {
    TVar r(v);
    r.id = active_tape()->leaf();
    return r;
  }
};
inline double val(const TVar& x) { return x.v; }
inline TVar operator+(TVar a, TVar b) { return TVar::make(a.v + b.v, a.id, 1.0, b.id, 1.0); }
inline TVar operator-(TVar a, TVar b) { return TVar::make(a.v - b.v, a.id, 1.0, b.id, -1.0); }
inline TVar operator*(TVar a, TVar b) { return TVar::make(a.v * b.v, a.id, b.v, b.id, a.v); }
inline TVar operator/(TVar a, TVar b) {
  const double q = a.v / b.v;
  return TVar::make(q, a.id, 1.0 / b.v, b.id, -q / b.v);
}
inline TVar operator-(TVar a) { return TVar::make(-a.v, a.id, -1.0, -1, 0.0); }
inline TVar& operator+=(TVar& a, TVar b) { a = a + b; return a; }
inline TVar& operator-=(TVar& a, TVar b) { a = a - b; return a; }
inline TVar sqrt_(TVar x) {
  const double s = std::sqrt(x.v);
  return TVar::make(s, x.id, 0.5 / s, -1, 0.0);
}
inline TVar abs_(TVar x) { return (x.v < 0.0) ? -x : x; }
inline TVar min_(TVar a, TVar b) { return (b.v < a.v) ? b : a; }
inline TVar max_(TVar a, TVar b) { return (b.v > a.v) ? b : a; }
inline TVar exp_(TVar x) {
  const double e = std::exp(x.v);
  return TVar::make(e, x.id, e, -1, 0.0);
}
inline TVar log_(TVar x) { return TVar::make(std::log(x.v), x.id, 1.0 / x.v, -1, 0.0); }

template <class R>
inline R sq(R x) { return x * x; }

}  // namespace oracle
