// The 6-point degree-4 rule on a triangle (two orbits of three points,
// Strang and Fix), used for every pair of triangles that share no vertex
// (Sec. 5.1) and for the field off the surface; 1 / (4 pi) of the Green's
// function.
#pragma once

namespace bemtx {

constexpr double kA1 = 0.445948490915964886318329253883;
constexpr double kW1 = 0.223381589678011465944827736698;
constexpr double kA2 = 0.091576213509770743459571463402;
constexpr double kW2 = 0.109951743655321867388505596635;
constexpr double kInv4Pi = 0.0795774715459476678844418816863;

// Barycentric coordinate c of point q of the 6-point rule, and its weight
// (weights sum to one; multiply by the area).
__host__ __device__ constexpr double r6_bary(int q, int c)
{
    return q < 3 ? (c == q ? 1.0 - 2.0 * kA1 : kA1) : (c == q - 3 ? 1.0 - 2.0 * kA2 : kA2);
}
__host__ __device__ constexpr double r6_w(int q) { return q < 3 ? kW1 : kW2; }

}  // namespace bemtx
