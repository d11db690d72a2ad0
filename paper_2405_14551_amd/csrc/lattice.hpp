// Velocity sets of the device path (D2Q9, D3Q19, D3Q27).
//
// Weights w_i are those of the second-order equilibrium (paper: Eq. disteq,
// c_s^2 = 1/3).  The D2Q9 numbering is the one the paper's periodic copy rules
// and Zou-He wall equations use (Sec. III.D): 1/3 = +-x, 2/4 = +-y, 5 = (+1,+1),
// 6 = (-1,+1), 7 = (-1,-1), 8 = (+1,-1).  The 3D sets list the rest velocity,
// then the six faces, twelve edges and eight corners in (+v, -v) pairs; D3Q19
// is the first 19 entries of D3Q27.  The perturbation coefficients are
// B_0 = w_0 - 2/3 and B_i = w_i, one exact solution of the isotropy
// constraints sum B = 1/3, sum B c = 0, sum B c c = I/3 (Sec. III.C.1).
//
// All tables are constexpr so that fully unrolled direction loops fold every
// c_i, w_i and opposite index into immediates.
#pragma once

namespace lbm {

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int cx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int cz[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  static constexpr int opp[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
  static constexpr double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                                  1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
};

struct D3Q27 {
  static constexpr int Q = 27;
  static constexpr int D = 3;
  //                          0   1   2  3   4  5   6  7   8  9  10 11  12 13  14 15  16 17  18 19  20 21  22 23  24  25 26
  static constexpr int cx[27] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, -1, 1};
  static constexpr int cy[27] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, -1, 1, 1, -1};
  static constexpr int cz[27] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, -1, 1, 1, -1, 1, -1};
  static constexpr int opp[27] = {0,  2,  1,  4,  3,  6,  5,  8,  7,  10, 9,  12, 11, 14,
                                  13, 16, 15, 18, 17, 20, 19, 22, 21, 24, 23, 26, 25};
  static constexpr double W0 = 8.0 / 27.0, W1 = 2.0 / 27.0, W2 = 1.0 / 54.0, W3 = 1.0 / 216.0;
  static constexpr double w[27] = {W0, W1, W1, W1, W1, W1, W1, W2, W2, W2, W2, W2, W2, W2,
                                   W2, W2, W2, W2, W2, W3, W3, W3, W3, W3, W3, W3, W3};
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int cx[19] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
  static constexpr int cy[19] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
  static constexpr int cz[19] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
  static constexpr int opp[19] = {0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17};
  static constexpr double W0 = 1.0 / 3.0, W1 = 1.0 / 18.0, W2 = 1.0 / 36.0;
  static constexpr double w[19] = {W0, W1, W1, W1, W1, W1, W1, W2, W2, W2,
                                   W2, W2, W2, W2, W2, W2, W2, W2, W2};
};

// first member of velocity pair p (its opposite is L::opp of it); pairs cover
// every moving direction once
template <class L>
constexpr int pair_first(int p) {
  if constexpr (L::D == 2) {
    constexpr int f[4] = {1, 2, 5, 6};
    return f[p];
  } else {
    return 2 * p + 1;
  }
}

template <class L>
constexpr double B_coef(int i) {
  return i == 0 ? L::w[0] - 2.0 / 3.0 : L::w[i];
}

template <class L>
constexpr int c2(int i) {
  return L::cx[i] * L::cx[i] + L::cy[i] * L::cy[i] + L::cz[i] * L::cz[i];
}

// 1/|c_i| (0 for the rest velocity)
template <class L>
constexpr double inv_norm(int i) {
  return c2<L>(i) == 0 ? 0.0 : (c2<L>(i) == 1 ? 1.0 : (c2<L>(i) == 2 ? 0.70710678118654752440 : 0.57735026918962576451));
}

}  // namespace lbm
