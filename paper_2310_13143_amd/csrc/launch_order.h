// Order in which the workgroups of a sweep launch take their blocks.
// Host and device code (the host build checks the mapping in CPU tests).
//
// The chip dispatches the workgroups of a launch to its 8 XCDs in turn
// (workgroup b to XCD b mod 8), and each XCD has its own L2.  When n blocks
// are used and the launch has at least 8 * ceil(n / 8) workgroups (xcd_grid),
// workgroup b takes the logical block (b mod 8) * ceil(n / 8) + b / 8: XCD x
// runs the contiguous logical blocks [x * per, (x + 1) * per), so that
// neighbouring blocks share an L2 (item blocks next to each other in bus
// order share the records of the lines between them, line blocks the values
// of nearby buses).  Every logical block below n is taken by exactly one
// workgroup; the others get -1 and exit.
#pragma once

#include "small_linalg.h"

namespace acopf {

constexpr int kXcds = 8;

ACOPF_HD int xcd_block(int b, int n) {
  const int per = (n + kXcds - 1) / kXcds;
  const int k = b / kXcds;
  if (k >= per) return -1;
  const int r = (b % kXcds) * per + k;
  return r < n ? r : -1;
}

// Workgroups to launch for a bound of n blocks: n rounded up to a multiple
// of 8.
inline unsigned xcd_grid(long long n) { return (unsigned)((n + kXcds - 1) / kXcds * kXcds); }

}  // namespace acopf
