// oracle_flops.cpp -- floating-point operation count of the oracle's
// right-hand-side expressions, per grid point.
//
// Test infrastructure: compiles the oracle's C source once more, as C++, with
// its floating-point type replaced by a tracing number.  Evaluating the
// oracle's right-hand side at one interior point then records every
// arithmetic operation in a tape (an expression graph whose leaves are the
// grid values the stencils read).  Reported, for the operations on which an
// output depends:
//   raw   -- as the oracle's code evaluates them (recomputation included);
//   cse   -- after merging identical operations on identical operands
//            (value numbering, the count of the expression itself);
// each split into the linear stencil part (differences and weights of grid
// values: the finite-difference operators) and the pointwise rest.
// Operations whose operands are all constants (grid spacings, weights) are
// folded; x+0, x-0, x*1, x/1 and x*0 are identities, negation is free (it
// folds into the neighbouring add or FMA on the hardware).  Every other
// +, -, *, / counts 1; sqrt, cbrt, exp, log, pow, sin, cos are listed apart.
//
// Usage: oracle_flops SYSTEM [fd_order] [slicing] [shift]
//   SYSTEM = wave | wave5 | bssn; prints one JSON object.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include <omp.h>

// built without OpenMP: the traced evaluation runs on one thread
extern "C" int omp_get_max_threads(void) { return 1; }

namespace tr {

enum Op { CONST, LEAF, ADD, SUB, MUL, DIV, NEG, SQRT, CBRT, EXP, LOG, POW, SIN, COS, NOPS };
const char* kName[NOPS] = {"const", "leaf", "add", "sub", "mul", "div", "neg",
                           "sqrt",  "cbrt", "exp", "log", "pow", "sin", "cos"};

struct Node {
  int op, a, b;
  double v;
};

std::vector<Node> tape(1, Node{CONST, 0, 0, 0.0});  // id 0 is never used
bool cse = true;
std::map<std::tuple<int, int, int>, int> seen;
std::map<double, int> consts;

int push(int op, int a, int b, double v) {
  if (cse && op != LEAF && op != CONST) {
    auto key = std::make_tuple(op, a, b);
    auto it = seen.find(key);
    if (it != seen.end()) return it->second;
    tape.push_back(Node{op, a, b, v});
    seen[key] = (int)tape.size() - 1;
    return (int)tape.size() - 1;
  }
  tape.push_back(Node{op, a, b, v});
  return (int)tape.size() - 1;
}

int constant(double v) {
  auto it = consts.find(v);
  if (it != consts.end()) return it->second;
  tape.push_back(Node{CONST, 0, 0, v});
  return consts[v] = (int)tape.size() - 1;
}

void reset(bool with_cse) {
  tape.assign(1, Node{CONST, 0, 0, 0.0});
  seen.clear();
  consts.clear();
  cse = with_cse;
}

struct Num {
  double v;
  int id;  // 0: an untracked constant (materialised on first use)
  Num() : v(0.0), id(0) {}
  template <class A, class = typename std::enable_if<std::is_arithmetic<A>::value>::type>
  Num(A x) : v((double)x), id(0) {}
  explicit operator double() const { return v; }
  explicit operator int() const { return (int)v; }
  explicit operator long() const { return (long)v; }
  explicit operator std::size_t() const { return (std::size_t)v; }
};

int node(const Num& x) { return x.id ? x.id : constant(x.v); }
bool is_const(const Num& x) { return x.id == 0 || tape[x.id].op == CONST; }
Num make(double v, int id) {
  Num r;
  r.v = v;
  r.id = id;
  return r;
}
Num leaf(double v) { return make(v, push(LEAF, 0, 0, v)); }

Num binary(int op, const Num& x, const Num& y, double v) {
  if (is_const(x) && is_const(y)) return Num(v);
  int a = node(x), b = node(y);
  if ((op == ADD || op == MUL) && a > b) std::swap(a, b);
  return make(v, push(op, a, b, v));
}

Num unary(int op, const Num& x, double v) {
  if (is_const(x)) return Num(v);
  return make(v, push(op, node(x), 0, v));
}

Num operator-(const Num& x) { return unary(NEG, x, -x.v); }
Num operator+(const Num& x) { return x; }
Num operator+(const Num& x, const Num& y) {
  if (is_const(y) && y.v == 0.0) return x;
  if (is_const(x) && x.v == 0.0) return y;
  return binary(ADD, x, y, x.v + y.v);
}
Num operator-(const Num& x, const Num& y) {
  if (is_const(y) && y.v == 0.0) return x;
  if (is_const(x) && x.v == 0.0) return -y;
  return binary(SUB, x, y, x.v - y.v);
}
Num operator*(const Num& x, const Num& y) {
  if ((is_const(x) && x.v == 0.0) || (is_const(y) && y.v == 0.0)) return Num(0.0);
  if (is_const(y) && y.v == 1.0) return x;
  if (is_const(x) && x.v == 1.0) return y;
  if (is_const(y) && y.v == -1.0) return -x;
  if (is_const(x) && x.v == -1.0) return -y;
  return binary(MUL, x, y, x.v * y.v);
}
Num operator/(const Num& x, const Num& y) {
  if (is_const(y) && y.v == 1.0) return x;
  if (is_const(x) && x.v == 0.0) return Num(0.0);
  return binary(DIV, x, y, x.v / y.v);
}
Num& operator+=(Num& x, const Num& y) { return x = x + y; }
Num& operator-=(Num& x, const Num& y) { return x = x - y; }
Num& operator*=(Num& x, const Num& y) { return x = x * y; }
Num& operator/=(Num& x, const Num& y) { return x = x / y; }
bool operator<(const Num& x, const Num& y) { return x.v < y.v; }
bool operator>(const Num& x, const Num& y) { return x.v > y.v; }
bool operator<=(const Num& x, const Num& y) { return x.v <= y.v; }
bool operator>=(const Num& x, const Num& y) { return x.v >= y.v; }
bool operator==(const Num& x, const Num& y) { return x.v == y.v; }
bool operator!=(const Num& x, const Num& y) { return x.v != y.v; }

Num sqrt(const Num& x) { return unary(SQRT, x, std::sqrt(x.v)); }
Num cbrt(const Num& x) { return unary(CBRT, x, std::cbrt(x.v)); }
Num exp(const Num& x) { return unary(EXP, x, std::exp(x.v)); }
Num log(const Num& x) { return unary(LOG, x, std::log(x.v)); }
Num sin(const Num& x) { return unary(SIN, x, std::sin(x.v)); }
Num cos(const Num& x) { return unary(COS, x, std::cos(x.v)); }
Num pow(const Num& x, const Num& y) { return binary(POW, x, y, std::pow(x.v, y.v)); }
Num fabs(const Num& x) { return x.v < 0 ? -x : x; }
Num floor(const Num& x) { return Num(std::floor(x.v)); }

}  // namespace tr

using tr::Num;
using tr::sqrt;
using tr::cbrt;
using tr::exp;
using tr::log;
using tr::sin;
using tr::cos;
using tr::pow;
using tr::fabs;
using tr::floor;

// the oracle, with its floating-point type traced
#define double Num
#include "../../oracle/oracle.c"
#undef double

namespace {

struct Count {
  long ops[tr::NOPS] = {};
  long linear = 0;  // live arithmetic operations of the stencil (linear) part
  long total() const {
    return ops[tr::ADD] + ops[tr::SUB] + ops[tr::MUL] + ops[tr::DIV];
  }
};

// live operations reachable from the outputs; linear = built only from grid
// values by +, -, negation, and products / quotients with constants
Count count_live(const std::vector<int>& outputs) {
  using namespace tr;
  std::vector<char> live(tape.size(), 0), lin(tape.size(), 0);
  std::vector<int> stack;
  for (int o : outputs)
    if (o) stack.push_back(o);
  while (!stack.empty()) {
    const int i = stack.back();
    stack.pop_back();
    if (live[i]) continue;
    live[i] = 1;
    const Node& n = tape[i];
    if (n.op != CONST && n.op != LEAF) {
      stack.push_back(n.a);
      if (n.op == ADD || n.op == SUB || n.op == MUL || n.op == DIV || n.op == POW)
        stack.push_back(n.b);
    }
  }
  Count c;
  for (size_t i = 1; i < tape.size(); i++) {  // operands precede results in the tape
    const Node& n = tape[i];
    auto L = [&](int j) { return lin[j] || tape[j].op == CONST; };
    auto C = [&](int j) { return tape[j].op == CONST; };
    switch (n.op) {
      case LEAF: lin[i] = 1; break;
      case ADD: case SUB: lin[i] = L(n.a) && L(n.b); break;
      case NEG: lin[i] = lin[n.a]; break;
      case MUL: lin[i] = (lin[n.a] && C(n.b)) || (C(n.a) && lin[n.b]); break;
      case DIV: lin[i] = lin[n.a] && C(n.b); break;
      default: lin[i] = 0;
    }
    if (!live[i]) continue;
    c.ops[n.op]++;
    if (lin[i] && (n.op == ADD || n.op == SUB || n.op == MUL || n.op == DIV)) c.linear++;
  }
  return c;
}

// pseudo-random smooth-ish positive data, so that no grid value is an exact
// constant the folding rules could act on
double datum(long i, int v) {
  const double x = std::sin(0.37 * (double)i + 1.3 * v) * 0.01;
  return (v == 0 || v == 17) ? 1.0 + x : x + 0.001 * (v + 1);  // chi, alpha near 1
}

Count run(const std::string& system, int order, int slicing, int shift, bool with_cse) {
  tr::reset(with_cse);
  orc_params p;
  std::memset(static_cast<void*>(&p), 0, sizeof p);
  for (int d = 0; d < 3; d++) {
    p.n[d] = 1;
    p.h[d] = Num(0.05 * (d + 1));
  }
  p.g = order == 8 ? 5 : (order == 6 ? 4 : 3);
  p.slicing = slicing;
  p.shift = shift;
  p.shift_F = Num(0.75);
  p.eta = Num(2.0);
  p.fd_order = order;
  const int nvar = system == "wave" ? 2 : (system == "wave5" ? 5 : 24);
  const geom G = mkgeom(&p);
  std::vector<Num> y(nvar * G.npts), r(nvar * G.npts);
  for (int v = 0; v < nvar; v++)
    for (long i = 0; i < G.npts; i++) y[v * G.npts + i] = tr::leaf(datum(i, v));
  if (system == "wave")
    orc_wave_rhs(&p, y.data(), r.data());
  else if (system == "wave5")
    orc_wave5_rhs(&p, y.data(), r.data());
  else
    orc_bssn_rhs(&p, y.data(), r.data());
  const long q = idx(&G, 0, 0, 0);
  std::vector<int> outs;
  for (int v = 0; v < nvar; v++) outs.push_back(r[v * G.npts + q].id);
  return count_live(outs);
}

void print(const char* key, const Count& c, bool last) {
  std::printf("\"%s\": {\"flops\": %ld, \"stencil\": %ld, \"pointwise\": %ld", key, c.total(),
              c.linear, c.total() - c.linear);
  for (int k = tr::ADD; k < tr::NOPS; k++)
    if (k != tr::NEG) std::printf(", \"%s\": %ld", tr::kName[k], c.ops[k]);
  std::printf("}%s", last ? "" : ", ");
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: %s wave|wave5|bssn [fd_order] [slicing] [shift]\n", argv[0]);
    return 2;
  }
  const std::string system = argv[1];
  const int order = argc > 2 ? std::atoi(argv[2]) : 4;
  const int slicing = argc > 3 ? std::atoi(argv[3]) : 0;
  const int shift = argc > 4 ? std::atoi(argv[4]) : 1;
  if (system != "wave" && system != "wave5" && system != "bssn") return 2;
  const Count raw = run(system, order, slicing, shift, false);
  const Count cse = run(system, order, slicing, shift, true);
  std::printf("{");
  print("raw", raw, false);
  print("cse", cse, true);
  std::printf("}\n");
  return 0;
}
