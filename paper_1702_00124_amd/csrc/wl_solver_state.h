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
  CG_RROLD = 10, // |r|^2 at the start of the iteration (the fused update keeps it for beta)
  CG_NROWS = 11
};
static_assert(CG_NROWS * 16 <= 256, "CG state rows overlap the multi-shift state");

// Multi-shift CG state (after the CG rows): per shifted system q = s * nrhs + r
// rows of kMaxSys doubles, then per-rhs rows of kMaxRhs.
constexpr int kMaxSys = 64;
constexpr int kMsState = 1280;  // offset in the device scalar area
enum MsStateRow {
  MS_ZPREV = 0,   // zeta_{i-1}
  MS_ZCUR = 1,    // zeta_i
  MS_ZNEXT = 2,   // zeta_{i+1}
  MS_ASHIFT = 3,  // alpha of the shifted system this iteration (0: frozen)
  MS_DONE = 4,    // 1 once |zeta|^2 |r|^2 <= tol^2 |b|^2
  MS_DELTA = 5,   // shift minus the base shift
  MS_ITERS = 6,   // base iterations when the system froze
  MS_NROWS = 7
};
constexpr int kMsRhsRows = kMsState + MS_NROWS * kMaxSys;  // per-rhs rows follow
enum MsRhsRow { MS_APREV = 0, MS_RHS_NROWS = 1 };

}  // namespace wl
