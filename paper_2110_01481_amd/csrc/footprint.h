// The line-model footprint of a unit pixel on the detector, shared by the strip-model
// projectors (forward and transpose).
#pragma once

#include "geometry.h"

namespace abg {
namespace {

// For an angle with p = max(|cos|,|sin|), q = min(...), the length of a line inside a
// unit pixel at distance t from its centre (detector units) is a trapezoid: 1/p for
// |t| <= h0 = (p-q)/2, falling linearly to 0 at h1 = (p+q)/2 (a box of width 1 when
// q = 0). Its integral from -inf to -a (a >= 0), times 1/ds, gives the strip model: the
// area of a pixel inside a strip of width ds at distance e from its centre is
//     G(e + ds/2) - G(e - ds/2),   G the antiderivative (total area 1).
template <typename T> struct Trapezoid {
    T h0, h1, i2pq, q2p, invp, hds, invds;
    Trapezoid() = default;
    __device__ Trapezoid(const AngleParams &P, double ds)
        : h0(T(P.p - P.half)), h1(T(P.half)), i2pq(T(0.5 * P.invpq)), q2p(T(0.5 * P.q * P.len)),
          invp(T(P.len)), hds(T(0.5 * ds)), invds(T(1.0 / ds))
    {
    }
    __device__ T below(T a) const
    {
        const T r = h1 - a;
        const T ramp = r * r * i2pq;
        const T flat = fma(h0 - a, invp, q2p);
        return a >= h1 ? T(0) : (a >= h0 ? ramp : flat);
    }
    // strip weight of a pixel whose centre is e >= 0 away from the ray (detector units)
    __device__ T strip(T e) const
    {
        const T lo = e - hds, hi = e + hds;
        const T glo = lo >= T(0) ? below(lo) : T(1) - below(-lo);
        return (glo - below(hi)) * invds;
    }
};

}  // namespace
}  // namespace abg
