// Instrumented operation count of the oracle: the oracle body compiled a third
// time with REAL = a counting type, so every floating-point add, subtract,
// multiply, divide, negation, exp and expm1 of one right-hand side evaluation
// (one cell-step) and of one gap-junction pair term is tallied. Test
// infrastructure: built and run by tests/test_oracle_pins.py only.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "../../oracle/infoli_oracle.c"

namespace {
long g_ops = 0;   // arithmetic operations
long g_tr = 0;    // of them, exp / expm1 calls
}

struct CReal {
    double v;
    CReal() : v(0.0) {}
    CReal(double x) : v(x) {}
};
static CReal operator+(CReal a, CReal b) { ++g_ops; return a.v + b.v; }
static CReal operator-(CReal a, CReal b) { ++g_ops; return a.v - b.v; }
static CReal operator*(CReal a, CReal b) { ++g_ops; return a.v * b.v; }
static CReal operator/(CReal a, CReal b) { ++g_ops; return a.v / b.v; }
static CReal operator-(CReal a) { ++g_ops; return -a.v; }
static CReal& operator+=(CReal& a, CReal b) { ++g_ops; a.v += b.v; return a; }
static bool operator==(CReal a, CReal b) { return a.v == b.v; }
static bool operator>(CReal a, CReal b) { return a.v > b.v; }
static bool operator<(CReal a, CReal b) { return a.v < b.v; }
static bool operator>=(CReal a, CReal b) { return a.v >= b.v; }
static bool operator<=(CReal a, CReal b) { return a.v <= b.v; }
static bool operator!=(CReal a, CReal b) { return a.v != b.v; }
static CReal count_exp(CReal a) { ++g_ops; ++g_tr; return std::exp(a.v); }
static CReal count_expm1(CReal a) { ++g_ops; ++g_tr; return std::expm1(a.v); }

#define REAL CReal
#define SFX(name) name##_cnt
#define EXP count_exp
#define EXPM1 count_expm1
#include "../../oracle/oracle_body.inc"

int main() {
    double pd[ORC_P], xd[ORC_S];
    // the default parameter table is passed on the command line (20 values)
    // so that this program holds no copy of it
    for (int k = 0; k < ORC_P; ++k) pd[k] = 0.0;
    for (int k = 0; k < ORC_P && std::scanf("%lf", &pd[k]) == 1; ++k) {}
    orc_rest_f64(pd, -60.0, xd);
    CReal p[ORC_P], x[ORC_S], dx[ORC_S];
    for (int k = 0; k < ORC_P; ++k) p[k] = pd[k];
    for (int k = 0; k < ORC_S; ++k) x[k] = xd[k];
    g_ops = g_tr = 0;
    orc_rhs_cnt(p, x, CReal(0.5), CReal(1.0), dx);
    const long rhs_ops = g_ops, rhs_tr = g_tr;
    g_ops = g_tr = 0;
    CReal t = pair_term_cnt(CReal(0.04), CReal(-60.0), CReal(-61.5));
    (void)t;
    std::printf("%ld %ld %ld %ld\n", rhs_ops, rhs_tr, g_ops, g_tr);
    return 0;
}
