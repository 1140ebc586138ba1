// lbm_stencil.hpp -- difference operators of Sec 2.3 for the gfx950 step.
#pragma once

#include <hip/hip_runtime.h>

namespace lbm {

enum Scheme { CD2 = 0, CD4 = 1, CD6 = 2, E4 = 3, E8 = 4, OCFDS4 = 5, CFDS4 = 6, CFDS6 = 7, CFDS8 = 8,
              E6 = 9, E10 = 10 };

__host__ __device__ constexpr bool is_compact(int s) { return s >= OCFDS4 && s <= CFDS8; }
__host__ __device__ constexpr bool is_iso(int s) { return s == E4 || s == E6 || s == E8 || s == E10; }

// Stencil radius of the explicit operators (compact schemes: radius of the
// right-hand side of Eq 21).
__host__ __device__ constexpr int radius(int s)
{
    return s == CD2 ? 1 : s == CD4 ? 2 : s == CD6 ? 3 : s == E4 ? 1 : s == E6 ? 2 : s == E8 ? 2 : 3;
}

// Explicit central first derivative, Eq 18-20: f' = sum_m d1(m) (f[+m] - f[-m]).
__host__ __device__ constexpr double d1(int s, int m)
{
    return s == CD2 ? (m == 1 ? 0.5 : 0.0)
         : s == CD4 ? (m == 1 ? 8.0 / 12.0 : m == 2 ? -1.0 / 12.0 : 0.0)
         : (m == 1 ? 45.0 / 60.0 : m == 2 ? -9.0 / 60.0 : m == 3 ? 1.0 / 60.0 : 0.0);
}

// Matched-order central second derivative (the Laplacian the paper leaves
// unstated for the explicit schemes): f'' = d2(0) f0 + sum_m d2(m)(f[+m] + f[-m]).
__host__ __device__ constexpr double d2(int s, int m)
{
    return s == CD2 ? (m == 0 ? -2.0 : m == 1 ? 1.0 : 0.0)
         : s == CD4 ? (m == 0 ? -30.0 / 12.0 : m == 1 ? 16.0 / 12.0 : m == 2 ? -1.0 / 12.0 : 0.0)
         : (m == 0 ? -490.0 / 180.0 : m == 1 ? 270.0 / 180.0 : m == 2 ? -27.0 / 180.0
            : m == 3 ? 2.0 / 180.0 : 0.0);
}

// Isotropic weights w(|e|^2) of Eq 25.  E4 in 2D as printed in Sec 2.3.3; in 3D
// the D3Q19 weights divided by cs^2.  E6, E8, E10 (the higher isotropy orders
// of Fig 6): the weights for which sum_i w (e_i.n)^(2m) is a multiple of
// |n|^(2m) for every 2m up to the order, with sum_i w e_ix^2 = 1, on the
// shells |e|^2 = 1,2,4 (E6, 2D), 1,2,3,4 (E6, 3D), 1,2,4,5,8 (E8, 2D),
// 1,2,3,4,5,6,8 (E8, 3D) and 1,2,4,5,8,9,10 (E10, 2D only).
__host__ __device__ constexpr double iso_w(int dim, int s, int sh)
{
    if (s == E4)
        return dim == 2 ? (sh == 1 ? 1.0 / 3.0 : sh == 2 ? 1.0 / 12.0 : 0.0)
                        : (sh == 1 ? 1.0 / 6.0 : sh == 2 ? 1.0 / 12.0 : 0.0);
    if (s == E6)
        return dim == 2 ? (sh == 1 ? 4.0 / 15.0 : sh == 2 ? 1.0 / 10.0 : sh == 4 ? 1.0 / 120.0 : 0.0)
                        : (sh == 1 ? 2.0 / 15.0 : sh == 2 ? 1.0 / 15.0 : sh == 3 ? 1.0 / 60.0
                           : sh == 4 ? 1.0 / 120.0 : 0.0);
    if (s == E10)
        return sh == 1 ? 262.0 / 1785.0 : sh == 2 ? 93.0 / 1190.0 : sh == 4 ? 7.0 / 340.0
             : sh == 5 ? 6.0 / 595.0 : sh == 8 ? 9.0 / 9520.0 : sh == 9 ? 2.0 / 5355.0
             : sh == 10 ? 1.0 / 7140.0 : 0.0;
    return dim == 2 ? (sh == 1 ? 4.0 / 21.0 : sh == 2 ? 4.0 / 45.0 : sh == 4 ? 1.0 / 60.0
                       : sh == 5 ? 2.0 / 315.0 : sh == 8 ? 1.0 / 5040.0 : 0.0)
                    : (sh == 1 ? 4.0 / 45.0 : sh == 2 ? 1.0 / 21.0 : sh == 3 ? 2.0 / 105.0
                       : sh == 4 ? 5.0 / 504.0 : sh == 5 ? 1.0 / 315.0 : sh == 6 ? 1.0 / 630.0
                       : sh == 8 ? 1.0 / 5040.0 : 0.0);
}

// Compact tridiagonal schemes, Eq 21 with beta = 0:
//   al f'_{i-1} + f'_i + al f'_{i+1} = ca (f_{i+1}-f_{i-1})/2 + cb (f_{i+2}-f_{i-2})/4
//                                      + cc (f_{i+3}-f_{i-3})/6.
// OCFDS4 (Sec 3.1) keeps the printed alpha and c; a and b follow from the two
// fourth-order conditions a + b + c = 1 + 2 alpha, a + 4b + 9c = 6 alpha.
struct Compact { double al, ca, cb, cc; };

inline Compact compact_scheme(int s)
{
    switch (s) {
    case CFDS4: return { 0.25, 1.5, 0.0, 0.0 };                          // Eq 22
    case CFDS6: return { 1.0 / 3.0, 14.0 / 9.0, 1.0 / 9.0, 0.0 };        // Eq 23
    case CFDS8: return { 3.0 / 8.0, 25.0 / 16.0, 1.0 / 5.0, -1.0 / 80.0 };  // Eq 24
    default: {
        const double al = 0.446776, c = -0.0541132;
        const double b = (4.0 * al - 1.0 - 8.0 * c) / 3.0;
        return { al, 1.0 + 2.0 * al - b - c, b, c };
    }
    }
}

}  // namespace lbm
