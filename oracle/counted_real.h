// Test infrastructure (oracle only): a double that counts its arithmetic.
//
// The oracle source is written against the scalar type `real`.  The normal
// build maps it to double; the counting build (-DORC_COUNT_FLOPS) maps it to
// CountedReal so that one run of the unchanged oracle reports how many FP64
// operations the method needs per face and per cell.  +, -, *, / and sqrt
// each count one operation; comparisons, min/max and fabs count none; pow and
// atan2 count one.  The counter is process global: run the counting build on
// one OpenMP thread.
#pragma once
#include <cmath>

extern long long g_orc_flops;

struct CountedReal {
  double v;
  CountedReal() : v(0.0) {}
  CountedReal(double x) : v(x) {}  // NOLINT: implicit on purpose
  explicit operator double() const { return v; }
  CountedReal& operator+=(CountedReal o) { ++g_orc_flops; v += o.v; return *this; }
  CountedReal& operator-=(CountedReal o) { ++g_orc_flops; v -= o.v; return *this; }
  CountedReal& operator*=(CountedReal o) { ++g_orc_flops; v *= o.v; return *this; }
  CountedReal& operator/=(CountedReal o) { ++g_orc_flops; v /= o.v; return *this; }
};
inline CountedReal operator+(CountedReal a, CountedReal b) { ++g_orc_flops; return CountedReal(a.v + b.v); }
inline CountedReal operator-(CountedReal a, CountedReal b) { ++g_orc_flops; return CountedReal(a.v - b.v); }
inline CountedReal operator*(CountedReal a, CountedReal b) { ++g_orc_flops; return CountedReal(a.v * b.v); }
inline CountedReal operator/(CountedReal a, CountedReal b) { ++g_orc_flops; return CountedReal(a.v / b.v); }
inline CountedReal operator-(CountedReal a) { return CountedReal(-a.v); }
inline bool operator<(CountedReal a, CountedReal b) { return a.v < b.v; }
inline bool operator>(CountedReal a, CountedReal b) { return a.v > b.v; }
inline bool operator<=(CountedReal a, CountedReal b) { return a.v <= b.v; }
inline bool operator>=(CountedReal a, CountedReal b) { return a.v >= b.v; }
inline bool operator==(CountedReal a, CountedReal b) { return a.v == b.v; }
inline bool operator!=(CountedReal a, CountedReal b) { return a.v != b.v; }
inline CountedReal sqrt(CountedReal a) { ++g_orc_flops; return CountedReal(std::sqrt(a.v)); }
inline CountedReal fabs(CountedReal a) { return CountedReal(std::fabs(a.v)); }
inline CountedReal pow(CountedReal a, CountedReal b) { ++g_orc_flops; return CountedReal(std::pow(a.v, b.v)); }
inline CountedReal atan2(CountedReal a, CountedReal b) { ++g_orc_flops; return CountedReal(std::atan2(a.v, b.v)); }
inline double to_double(CountedReal a) { return a.v; }
