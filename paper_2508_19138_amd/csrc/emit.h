// Emission of the RGF recursion as one lane's operation list.
#pragma once
#include "../../include/qtx_rgf.h"
#include "exec.h"

namespace qtx {

// Per-problem sizes and options fixed before lanes are built.
struct Plan {
  int n = 0, b = 0, ne = 0, nr = 0;
  bool is_w = false;
  bool general_ul = false;   // U/L assembled per energy
  bool need_hl = false;      // H.lower absent: H.upper^dagger built once
  bool bt_rhs[2] = {false, false};
  bool fp32 = false;
};

Plan make_plan(const qtx_rgf_problem& p);

// Exact workspace bytes of one lane of `ec` energies.
size_t lane_bytes(const Plan& q, int ec);

// Operations of one lane (energies e0 .. e0+ec-1 of problem p) whose
// workspace is ws[0 .. lane_bytes(q, ec)).  d_E: the problem's energies on
// the device (G-type), d_info: the problem's per-energy status words.  When
// H.lower is absent the lane builds its own H.upper^dagger first.
void build_lane(Lane& lane, const qtx_rgf_problem& p, const Plan& q, char* ws,
                int e0, int ec, const double* d_E, int* d_info, Tuner& tuner,
                hipStream_t s);

// Shape class of a problem's lanes: lanes of one class have the same
// operation sequence up to its length (block count) and the block size of
// its operands; size_key 2 also separates block sizes, 1 separates blocks
// up to 256 from larger ones, 0 neither.  Lanes of one class started
// together run in lockstep and share every launch.
uint64_t lane_class(const Plan& q, const qtx_rgf_problem& p, int size_key);

}  // namespace qtx
