/*
 * Op-counting build of the FP64 oracle (quadswarm_oracle.c).
 *
 * MEASUREMENT INFRASTRUCTURE ONLY, like the oracle itself: it gives the
 * algorithmic floating-point work of the method -- what the plain,
 * one-quad-at-a-time definition of a step, an observation or a reverse pass
 * computes -- so that a kernel's rate can be priced against the chip's
 * vector peak.  The oracle's source is compiled unchanged, as C++, with
 * every `double` replaced by or_num, a double that counts the arithmetic
 * done on it.  Results are bitwise those of the plain oracle (same IEEE
 * operations in the same order, no contraction).
 *
 * Counted: add/subtract, multiply, divide, square root, and the
 * transcendental functions (exp, log, log1p, sin, cos).  Not counted:
 * comparisons, negation, fabs, copies, and what the oracle marks with
 * OR_MARGIN (threshold-margin diagnostics) or OR_CONST (constants derived
 * from a quad's parameters, which the plain oracle recomputes every
 * substep although they are fixed per quad).
 *
 * The counters are global (the counting build is run single-threaded) and
 * read with or_opcount_get: [add, mul, div, sqrt, transcendental].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

namespace {
uint64_t g_count[5];  // add, mul, div, sqrt, transcendental
int g_paused = 0;
inline void tick(int k) {
  if (!g_paused) ++g_count[k];
}
}  // namespace

struct or_num {
  double v;
  or_num() = default;
  or_num(double x) : v(x) {}  // NOLINT: literals and casts convert implicitly
  or_num(int x) : v((double)x) {}
  or_num(unsigned x) : v((double)x) {}
  or_num(long x) : v((double)x) {}
  or_num(unsigned long x) : v((double)x) {}
  or_num(long long x) : v((double)x) {}
  or_num(unsigned long long x) : v((double)x) {}
  explicit operator double() const { return v; }
  or_num& operator+=(or_num b) { tick(0); v += b.v; return *this; }
  or_num& operator-=(or_num b) { tick(0); v -= b.v; return *this; }
  or_num& operator*=(or_num b) { tick(1); v *= b.v; return *this; }
  or_num& operator/=(or_num b) { tick(2); v /= b.v; return *this; }
};

inline or_num operator+(or_num a, or_num b) { tick(0); return or_num(a.v + b.v); }
inline or_num operator-(or_num a, or_num b) { tick(0); return or_num(a.v - b.v); }
inline or_num operator*(or_num a, or_num b) { tick(1); return or_num(a.v * b.v); }
inline or_num operator/(or_num a, or_num b) { tick(2); return or_num(a.v / b.v); }
inline or_num operator-(or_num a) { return or_num(-a.v); }
inline or_num operator+(or_num a) { return a; }
inline bool operator<(or_num a, or_num b) { return a.v < b.v; }
inline bool operator<=(or_num a, or_num b) { return a.v <= b.v; }
inline bool operator>(or_num a, or_num b) { return a.v > b.v; }
inline bool operator>=(or_num a, or_num b) { return a.v >= b.v; }
inline bool operator==(or_num a, or_num b) { return a.v == b.v; }
inline bool operator!=(or_num a, or_num b) { return a.v != b.v; }
inline bool operator!(or_num a) { return !a.v; }

inline or_num sqrt(or_num a) { tick(3); return or_num(::sqrt(a.v)); }
inline or_num exp(or_num a) { tick(4); return or_num(::exp(a.v)); }
inline or_num log(or_num a) { tick(4); return or_num(::log(a.v)); }
inline or_num log1p(or_num a) { tick(4); return or_num(::log1p(a.v)); }
inline or_num sin(or_num a) { tick(4); return or_num(::sin(a.v)); }
inline or_num cos(or_num a) { tick(4); return or_num(::cos(a.v)); }
inline or_num fabs(or_num a) { return or_num(::fabs(a.v)); }

// what the oracle marks is evaluated with the count paused
template <typename F>
inline auto uncounted(F&& f) {
  ++g_paused;
  auto r = f();
  --g_paused;
  return r;
}
#define OR_CONST(x) uncounted([&]() -> or_num { return (x); })
#define OR_MARGIN(mg, val) ((void)uncounted([&]() { upd_margin(mg, val); return 0; }))

extern "C" {
#define double or_num
#include "quadswarm_oracle.c"
#undef double

void or_opcount_reset(void) { memset(g_count, 0, sizeof(g_count)); }

void or_opcount_get(uint64_t out[5]) {
  for (int k = 0; k < 5; ++k) out[k] = g_count[k];
}
}
