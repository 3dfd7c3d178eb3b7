// Scan geometry of the projectors: per-angle constants (computed on the host in FP64) and
// the image / sinogram sizes.
#pragma once

#include <vector>

namespace abg {

// Zero columns on each side of the padded image copies read by the forward projector.
constexpr int kPad = 4;

// Per-angle constants, computed on the host in FP64 when the geometry is created.
struct AngleParams {
    double c, s;        // cos(theta), sin(theta); exact 0 / +-1 at multiples of 90 degrees
    double p, q;        // max(|c|,|s|), min(|c|,|s|)
    // ray-driven forward projector: the ray advances one pixel along its major axis
    // (rows when |c| >= |s|, columns otherwise) per step and moves `m` pixels along
    // the minor axis; it is 1/p long inside each major-axis band.
    double m;           // -s/c (steep) or -c/s (flat)
    double inv;         // 1/c (steep) or 1/s (flat)
    double len;         // 1/p
    double invq;        // 1/q (0 when q == 0)
    // pixel-driven back projectors: detector coordinate u = <c_j, omega>/ds - s0/ds
    double cu, su;      // cos/ds, sin/ds: change of u per pixel step in x and in y
    double half;        // (p+q)/2: half-width of the line-model trapezoid
    double invpq;       // 1/(p q) (0 when q == 0)
    int steep;          // 1: walk image rows, 0: walk image columns
    int axis;           // 1 when q == 0 (ray parallel to a pixel edge)
};

struct Geometry {
    int N = 0, n_ang = 0, n_det = 0;
    double ds = 1.0;
    int model = 0;      // forward projector: ABG_FP_LINE, ABG_FP_STRIP or ABG_FP_JOSEPH
    // thresholded strip back projector B_tau: entries below tau_thr are dropped
    double strip_max = 0.0;   // largest strip-model entry (0: not computed yet)
    double tau_thr = -1.0;    // tau * strip_max - tie band (tau = 0: keep every entry)
    int device = 0;
    std::vector<double> theta;
    std::vector<AngleParams> host;
    AngleParams *dev = nullptr;
    // NCP periodogram tables (chirp transform of the row length), built on first use
    mutable void *ncp_tab = nullptr;
    long long n() const { return (long long)N * N; }
    long long m() const { return (long long)n_ang * n_det; }
    int padded_stride() const { return N + 2 * kPad; }
};

}  // namespace abg
