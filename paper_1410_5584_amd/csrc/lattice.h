// Lattice descriptors for the device code: velocities, weights and the mode
// basis used by the noise back-transform and the mode observables.
//
// Weights follow from the isotropy relations of Eq. (77) with c_s^2 = 1/3
// (Sec. V B).  D2Q9 modes are Table I; D3Q19 modes are the Hermite modes of
// Eq. (26) plus nine ghosts chosen, as Sec. V B requires, only to keep the
// discrete orthogonality / completeness of Eq. (79) (the layout is spelled out
// in include/fmlb.h).  All entries are compile-time constants so that fully
// unrolled loops fold every zero and small integer away.
#pragma once

#include <hip/hip_runtime.h>

namespace fmlb {

struct D2Q9 {
    static constexpr int Q = 9;
    static constexpr int D = 2;
    static constexpr int NS = Q - D - 1;  // non-momentum, non-density modes per species
    static constexpr int cx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
    static constexpr int cy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    // weights in units of 1/36
    static constexpr int w36[Q] = {16, 4, 4, 4, 4, 1, 1, 1, 1};
    // Table I rows T_a(c_i), a = 0..8
    static constexpr int T[Q][Q] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1},            // rho
        {0, 1, 0, -1, 0, 1, -1, -1, 1},         // j_x
        {0, 0, 1, 0, -1, 1, 1, -1, -1},         // j_y
        {-2, 1, 1, 1, 1, 4, 4, 4, 4},           // e      = 3|c|^2 - 2
        {0, 1, -1, 1, -1, 0, 0, 0, 0},          // P_ww   = 2 c_x^2 - |c|^2
        {0, 0, 0, 0, 0, 1, -1, 1, -1},          // P_xy   = c_x c_y
        {0, -1, 0, 1, 0, 2, -2, -2, 2},         // q_x    = (3|c|^2 - 4) c_x
        {0, 0, -1, 0, 1, 2, 2, -2, -2},         // q_y    = (3|c|^2 - 4) c_y
        {2, -4, -4, -4, -4, 8, 8, 8, 8}};       // eps    = 9|c|^4 - 15|c|^2 + 2
    // squared norms N_a = sum_i w_i T_ai^2 as numerator / denominator
    static constexpr int Nnum[Q] = {1, 1, 1, 4, 4, 1, 2, 2, 16};
    static constexpr int Nden[Q] = {1, 3, 3, 1, 9, 9, 3, 3, 1};
};

struct D3Q19 {
    static constexpr int Q = 19;
    static constexpr int D = 3;
    static constexpr int NS = Q - D - 1;
    static constexpr int cx[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
    static constexpr int cy[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
    static constexpr int cz[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
    static constexpr int w36[Q] = {12, 2, 2, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    // Modes scaled by 3 where the Hermite form has thirds (3 T_a); the scale
    // of a mode does not change the collision (amplitudes scale with sqrt(N)).
    // Row a lists 3 T_a(c_i) for a = 4..6 and T_a(c_i) otherwise.
    static constexpr int T[Q][Q] = {
        {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
        {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
        {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
        {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
        // 3 c_x^2 - 1, 3 c_y^2 - 1, 3 c_z^2 - 1
        {-1, 2, 2, -1, -1, -1, -1, 2, 2, 2, 2, 2, 2, 2, 2, -1, -1, -1, -1},
        {-1, -1, -1, 2, 2, -1, -1, 2, 2, 2, 2, -1, -1, -1, -1, 2, 2, 2, 2},
        {-1, -1, -1, -1, -1, 2, 2, -1, -1, -1, -1, 2, 2, 2, 2, 2, 2, 2, 2},
        // c_x c_y, c_y c_z, c_x c_z
        {0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, -1, -1, 0, 0, 0, 0},
        // (3|c|^2 - 5) c_x, c_y, c_z
        {0, -2, 2, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0},
        {0, 0, 0, -2, 2, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1},
        {0, 0, 0, 0, 0, -2, 2, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1},
        // (c_y^2 - c_z^2) c_x, (c_z^2 - c_x^2) c_y, (c_x^2 - c_y^2) c_z
        {0, 0, 0, 0, 0, 0, 0, 1, -1, 1, -1, -1, 1, -1, 1, 0, 0, 0, 0},
        {0, 0, 0, 0, 0, 0, 0, -1, 1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1},
        {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 1, -1, -1, 1, -1, 1, 1, -1},
        // (2|c|^2 - 3)(3 c_x^2 - |c|^2), (2|c|^2 - 3)(c_y^2 - c_z^2)
        {0, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, -2, -2, -2, -2},
        {0, 0, 0, -1, -1, 1, 1, 1, 1, 1, 1, -1, -1, -1, -1, 0, 0, 0, 0},
        // 3|c|^4 - 6|c|^2 + 1
        {1, -2, -2, -2, -2, -2, -2, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1}};
    // squared norms of the rows above (the scaled rows 4..6 have 9 * 2/9 = 2)
    static constexpr int Nnum[Q] = {1, 1, 1, 1, 2, 2, 2, 1, 1, 1, 2, 2, 2, 2, 2, 2, 4, 4, 2};
    static constexpr int Nden[Q] = {1, 3, 3, 3, 1, 1, 1, 9, 9, 9, 3, 3, 3, 9, 9, 9, 3, 9, 1};
};

// Index of the velocity opposite to i.
template <class L>
__host__ __device__ constexpr int opposite(int i)
{
    for (int k = 0; k < L::Q; ++k)
        if (L::cx[k] == -L::cx[i] && L::cy[k] == -L::cy[i] && L::cz[k] == -L::cz[i]) return k;
    return -1;
}

}  // namespace fmlb
