// Layout of the device-resident CG state: rows of kMaxRhs doubles.
#pragma once

namespace wl {

enum CgStateRow {
  CG_RR = 0,     // |r|^2 of the current iterate
  CG_PAP = 1,    // <p, A p>
  CG_ALPHA = 2,
  CG_BETA = 3,
  CG_BB = 4,     // |b|^2
  CG_DONE = 5,   // 1 once |r|^2 <= tol^2 |b|^2 (iteration frozen)
  CG_ITERS = 6,
  CG_TOL2 = 7,
  CG_MAXRR = 8,  // largest |r|^2 since the last reliable update
  CG_BREAK = 9,  // set when <p, A p> or |r|^2 is not a positive finite number
  CG_NROWS = 10
};

}  // namespace wl
