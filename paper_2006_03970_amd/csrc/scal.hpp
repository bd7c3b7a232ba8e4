// Slots of the small device scalar buffer that the kernels fill and the host
// reads back at each synchronisation point (one copy per Newton iteration).
#pragma once

namespace ssnal {

enum Scal : int {
  SC_R = 0,      // |J|, written by the compaction pass
  SC_S = 1,      // accepted line-search step (0 when no trial passed)
  SC_LSK = 2,    // accepted trial index, -1 when none
  SC_GD = 3,     // <grad psi, d>
  SC_DD = 4,     // |d|^2
  SC_GG = 5,     // |grad psi|^2
  SC_RR = 6,     // |A x_new - b|^2
  SC_BR = 7,     // b^T (A x_new - b)
  SC_XU = 8,     // |x - u|^2 (multiplier update)
  SC_ZZ = 9,     // |z|^2
  SC_YY = 10,    // |y|^2
  SC_ETA_E = 11, // |x - prox_p(x - A^T rho)|^2
  SC_ETA_XX = 12,
  SC_ETA_X1 = 13,
  SC_ETA_PS = 14,  // sum (|q| - lambda1)_+^2, q = A^T rho
  SC_NONFIN = 15,  // count of non-finite entries
  SC_CHOL = 16,    // Cholesky status (0 or pivot+1), stored as double
  SC_AMAX = 17,    // max_i |v_i| (path: ||A^T b||_inf)
  SC_COLSQ = 18,   // sum_j ||a_j||^2 (default sigma0)
  SC_BB = 19,      // ||b||^2
  SC_MS_RSSEN = 20,  // model selection: ||A x - b||^2
  SC_MS_FROB = 21,   // ||L^{-1}||_F^2
  SC_MS_RSS = 22,    // ||A_J beta - b||^2
  SC_MS_NONE = 23,   // sink of an empty sum
  SC_CV_MT = 24,     // k-fold: training rows of the current fold
  SC_CV_MV = 25,     // validation rows of the current fold
  SC_CV_BAD = 26,    // fold labels outside [0, k)
  SC_CG_RR = 27,     // conjugate gradients: |res|^2, two slots by iteration parity
  SC_CG_STOP = 29,   // eps^2 |g|^2
  SC_CG_DONE = 30,   // 1 once |res|^2 <= stop
  SC_CG_IT = 31,     // iterations taken
  SC_DELTA = 32,   // 33 slots: line-search increments Delta_k (+ second-order sum)
  SC_BLK = 80,     // per-block partials of the m-vector finishers (<= 16 blocks x 3)
  SC_SIZE = 160
};
// Block partials (3 each) the scalar block holds from SC_BLK on: m <= 16 * 256.
constexpr int kScalBlocks = 16;

}  // namespace ssnal
