// D3Q19 lattice of the relativistic LB scheme (the model paragraph and
// Fig. 2: 19 velocities, the fastest sqrt(2) c_l; weights 1/3 rest, 1/18 for
// |c_i| = c_l, 1/36 for |c_i| = sqrt(2) c_l).  Ordering: rest; the six axis
// directions as (+,-) pairs; the twelve diagonals as (v, -v) pairs, so that
// the opposite of 2k-1 is 2k.
#pragma once

namespace rlb {

constexpr int Q = 19;

constexpr int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
constexpr int OPP[Q] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};

constexpr double W0 = 1.0 / 3.0;
constexpr double W1 = 1.0 / 18.0;
constexpr double W2 = 1.0 / 36.0;
constexpr double WQ[Q] = {W0, W1, W1, W1, W1, W1, W1, W2, W2, W2, W2,
                          W2, W2, W2, W2, W2, W2, W2, W2};

}  // namespace rlb
