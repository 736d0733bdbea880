// counted_double.hpp -- a double that counts the arithmetic done on it.
//
// TEST AND MEASUREMENT INFRASTRUCTURE.  Force-included (g++ -include) ahead of
// the oracle's C sources, compiled as C++, it replaces the oracle's `double`
// by `cdouble`, whose +, -, *, / and sqrt each add one to a global counter, so
// that running the unchanged oracle on a workload counts the floating-point
// operations of the method as the oracle states it.  Comparisons, |x|, min,
// max and sign changes are counted apart (they are not flops).  The values are
// those of plain double arithmetic: each operator applies the double operation
// once.
#pragma once
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <cmath>

namespace flopcount {
// [0] add/sub, [1] mul, [2] div, [3] sqrt, [4] compare/abs/min/max
extern uint64_t ops[5];
}

struct cdouble {
    double v;
    cdouble() = default;
    constexpr cdouble(double x) : v(x) {}
    explicit operator double() const { return v; }
    explicit operator int() const { return int(v); }
    explicit operator long long() const { return (long long)v; }
};

#define FC_BIN(OP, K)                                                                     \
    inline cdouble operator OP(cdouble a, cdouble b) { ++flopcount::ops[K]; return a.v OP b.v; } \
    inline cdouble operator OP(cdouble a, double b) { ++flopcount::ops[K]; return a.v OP b; }    \
    inline cdouble operator OP(double a, cdouble b) { ++flopcount::ops[K]; return a OP b.v; }    \
    inline cdouble &operator OP##=(cdouble &a, cdouble b) { ++flopcount::ops[K]; a.v = a.v OP b.v; return a; } \
    inline cdouble &operator OP##=(cdouble &a, double b) { ++flopcount::ops[K]; a.v = a.v OP b; return a; }
FC_BIN(+, 0)
FC_BIN(-, 0)
FC_BIN(*, 1)
FC_BIN(/, 2)
#undef FC_BIN
inline cdouble operator-(cdouble a) { return -a.v; }
inline cdouble operator+(cdouble a) { return a; }

#define FC_CMP(OP)                                                                   \
    inline bool operator OP(cdouble a, cdouble b) { ++flopcount::ops[4]; return a.v OP b.v; } \
    inline bool operator OP(cdouble a, double b) { ++flopcount::ops[4]; return a.v OP b; }    \
    inline bool operator OP(double a, cdouble b) { ++flopcount::ops[4]; return a OP b.v; }
FC_CMP(<)
FC_CMP(>)
FC_CMP(<=)
FC_CMP(>=)
FC_CMP(==)
FC_CMP(!=)
#undef FC_CMP

inline cdouble sqrt(cdouble a) { ++flopcount::ops[3]; return std::sqrt(a.v); }
inline cdouble fabs(cdouble a) { ++flopcount::ops[4]; return std::fabs(a.v); }
inline cdouble fmin(cdouble a, cdouble b) { ++flopcount::ops[4]; return std::fmin(a.v, b.v); }
inline cdouble fmax(cdouble a, cdouble b) { ++flopcount::ops[4]; return std::fmax(a.v, b.v); }
inline cdouble copysign(cdouble a, cdouble b) { return std::copysign(a.v, b.v); }
inline bool isfinite(cdouble a) { return std::isfinite(a.v); }
inline bool isnan(cdouble a) { return std::isnan(a.v); }

// the C sources assign malloc's result to typed pointers without a cast
struct fc_any_ptr {
    void *p;
    template <class T> operator T *() const { return static_cast<T *>(p); }
};
#define malloc(n) (fc_any_ptr{::malloc(n)})

#define double cdouble
