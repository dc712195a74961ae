// D2Q37 model constants for the GPU path.
//
// Velocity set (paper, Section 3 and Fig. 1): 37 populations per site, each
// hopping up to three lattice points. Here: every integer hop c with
// |c|^2 <= 10, ordered lexicographically in (cx, cy); the rest population is
// index 18 and the opposite of population i is 36 - i. The paper leaves the
// labels arbitrary; this order is the library's public population order
// (the canonical [37][LX][LY] interchange arrays use it).
//
// Weights and lattice scale: the unique positive solution of the moment
// conditions that make sum_i w_i q(r c_i) equal the integral of q against
// the unit Gaussian for every polynomial q of degree <= 9 (one weight per
// shell |c|^2 in {0,1,2,4,5,8,9,10}, plus theta = 1/r^2). The literals below
// are that solution, correctly rounded from 35 significant digits.
#pragma once

#include <cstdint>

namespace d2q37 {

constexpr int Q = 37;
constexpr int NPAIR = 18;  // populations 0..17 pair with 36..19; 18 is at rest
constexpr int REST = 18;
constexpr int NSHELL = 8;

// Hops, lexicographic in (cx, cy).
constexpr int CX[Q] = {-3, -3, -3, -2, -2, -2, -2, -2, -1, -1, -1, -1, -1, -1, -1, 0, 0, 0, 0,
                       0,  0,  0,  1,  1,  1,  1,  1,  1,  1,  2,  2,  2,  2,  2,  3, 3, 3};
constexpr int CY[Q] = {-1, 0, 1, -2, -1, 0, 1, 2, -3, -2, -1, 0, 1, 2, 3, -3, -2, -1, 0,
                       1,  2, 3, -3, -2, -1, 0, 1, 2, 3,  -2, -1, 0, 1, 2, -1, 0,  1};

constexpr int c2_of(int p) { return CX[p] * CX[p] + CY[p] * CY[p]; }

// Shell of each population: |c|^2 = 0,1,2,4,5,8,9,10 -> 0..7.
constexpr int shell_of_c2(int c2)
{
    return c2 == 0 ? 0 : c2 == 1 ? 1 : c2 == 2 ? 2 : c2 == 4 ? 3 : c2 == 5 ? 4 : c2 == 8 ? 5 : c2 == 9 ? 6 : 7;
}
constexpr int SHELL_C2[NSHELL] = {0, 1, 2, 4, 5, 8, 9, 10};

// Shell weights.
constexpr double WSH[NSHELL] = {
    0.23315066913235250228650670406684995,    // |c|^2 = 0
    0.10730609154221900241246428718313994,    // 1
    0.057667859888794882030069215393339415,   // 2
    0.014208216158450750264698942344134455,   // 4
    0.0053530490005137752327315016621884935,  // 5
    0.0010119375926735754754109085066391147,  // 8
    0.00024530102775771734546591664326784446, // 9
    0.00028341425299419821740052529419488023, // 10
};
// Lattice scale: thermal velocity xi = R * c; THETA = 1 / R^2.
constexpr double R = 1.1969797703930743589723884638532754;
constexpr double THETA = 0.69795332201968308823840905538932529;
constexpr double R2 = 1.4327605707302570117458414113090480;  // 1 / THETA

constexpr double weight(int p) { return WSH[shell_of_c2(c2_of(p))]; }

// FP16 storage scale per shell: an exact power of two close to 1 / w, so
// that g * s is O(|g / w|) and stays clear of FP16 subnormals.
constexpr float S16[NSHELL] = {4.0f, 8.0f, 16.0f, 64.0f, 256.0f, 1024.0f, 4096.0f, 4096.0f};

}  // namespace d2q37
