// sin and cos of the phase k r of the Helmholtz Green's function, FP64.
//
// Method: Cody-Waite reduction x = n (pi/2) + r with pi/2 split into three
// parts (33 + 33 + 53 significant bits, so that n * P1 and n * P2 are exact
// for |n| < 2^20) applied with fused multiply-adds, then Taylor polynomials
// of sin (through r^17) and cos (through r^16) on |r| <= pi/4, where the
// truncation error is below 1e-19, and quadrant selection from n mod 4.
// Valid for |x| < 1e5 (exact reduction); problems whose phases could exceed
// that are rejected when they are created.
// The split constants and the coefficients 1/n! were generated for this
// file from the decimal expansion of pi with exact rational arithmetic.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace bemtx {

constexpr double kPhaseMax = 1.0e5;   // largest |k r| the reduction is exact for

__host__ __device__ inline void phase_sincos(double x, double *s, double *c)
{
    constexpr double kTwoOverPi = 0.6366197723675814;
    constexpr double P1 = 1.5707963267341256;      // pi/2, leading 33 bits
    constexpr double P2 = 6.077100506303966e-11;   // next 33 bits
    constexpr double P3 = 2.0222662487959506e-21;  // remainder
    const double n = rint(x * kTwoOverPi);
    double r = fma(-n, P1, x);
    r = fma(-n, P2, r);
    r = fma(-n, P3, r);
    const double z = r * r;
    double ps = 2.8114572543455206e-15;            //  1/17!
    ps = fma(ps, z, -7.647163731819816e-13);       // -1/15!
    ps = fma(ps, z, 1.6059043836821613e-10);       //  1/13!
    ps = fma(ps, z, -2.505210838544172e-08);       // -1/11!
    ps = fma(ps, z, 2.7557319223985893e-06);       //  1/9!
    ps = fma(ps, z, -0.0001984126984126984);       // -1/7!
    ps = fma(ps, z, 0.008333333333333333);         //  1/5!
    ps = fma(ps, z, -0.16666666666666666);         // -1/3!
    const double sr = fma(r * z, ps, r);
    double pc = 4.779477332387385e-14;             //  1/16!
    pc = fma(pc, z, -1.1470745597729725e-11);      // -1/14!
    pc = fma(pc, z, 2.08767569878681e-09);         //  1/12!
    pc = fma(pc, z, -2.755731922398589e-07);       // -1/10!
    pc = fma(pc, z, 2.48015873015873e-05);         //  1/8!
    pc = fma(pc, z, -0.001388888888888889);        // -1/6!
    pc = fma(pc, z, 0.041666666666666664);         //  1/4!
    pc = fma(pc, z, -0.5);                         // -1/2!
    const double cr = fma(z, pc, 1.0);
    const int q = (int)n & 3;
    double sv = (q & 1) ? cr : sr;
    double cv = (q & 1) ? sr : cr;
    if (q & 2) sv = -sv;
    if ((q + 1) & 2) cv = -cv;
    *s = sv;
    *c = cv;
}

}  // namespace bemtx
