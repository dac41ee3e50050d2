// D3Q19 lattice constants for the device code.
//
// Velocity order (the library's canonical order): rest, +-x, +-y, +-z, then the twelve face
// diagonals, each followed by its opposite. Lattice weights 1/3, 1/18, 1/36 with c_s^2 = 1/3
// (Sec. 2 and Sec. 4 of arXiv:2105.08772 use D3Q19 with c_s^2 = 1/3). The Shan-Chen forcing
// weights of Eq. (SCForce), W(1) = 1/6 and W(2) = 1/12, equal w_i / c_s^2, so the force and the
// pressure tensor are written below with c_s^2 W = w.
#pragma once

namespace lbm {

constexpr int Q = 19;

constexpr int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
constexpr int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
constexpr int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

constexpr double W0 = 1.0 / 3.0;
constexpr double W1 = 1.0 / 18.0;
constexpr double W2 = 1.0 / 36.0;

constexpr double weight(int i) { return i == 0 ? W0 : (i <= 6 ? W1 : W2); }

}  // namespace lbm
