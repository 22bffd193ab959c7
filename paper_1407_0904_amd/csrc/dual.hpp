// Forward-mode dual numbers (value + one directional derivative) for the
// reverse pass of the assembly: the geometry and geometry-tensor code is
// templated on its scalar type and run on Dual to differentiate the per-cell
// functional with respect to each local input.
#pragma once
#include <hip/hip_runtime.h>

namespace coffee {
namespace dev {

struct Dual {
    double v, d;
    __device__ Dual() = default;
    __device__ constexpr Dual(double x) : v(x), d(0.0) {}
    __device__ constexpr Dual(double x, double dx) : v(x), d(dx) {}
    __device__ Dual& operator+=(const Dual& o) { v += o.v; d += o.d; return *this; }
    __device__ Dual& operator-=(const Dual& o) { v -= o.v; d -= o.d; return *this; }
    __device__ Dual& operator*=(const Dual& o) { d = d * o.v + v * o.d; v *= o.v; return *this; }
};

__device__ inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
__device__ inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
__device__ inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
__device__ inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
__device__ inline Dual operator/(Dual a, Dual b) { return Dual(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
__device__ inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
__device__ inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
__device__ inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
__device__ inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
__device__ inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
__device__ inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
__device__ inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
__device__ inline Dual operator/(double a, Dual b) { return Dual(a / b.v, -a * b.d / (b.v * b.v)); }

__host__ __device__ inline double absval(double x) { return fabs(x); }
__device__ inline Dual absval(Dual x) { return x.v < 0.0 ? -x : x; }
__device__ inline double value_of(double x) { return x; }
__device__ inline double value_of(Dual x) { return x.v; }

}  // namespace dev
}  // namespace coffee
