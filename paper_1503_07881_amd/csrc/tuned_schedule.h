// Generated from tuned_schedules.json by `python -m paper_1503_07881_amd.autotune --emit-header`;
// do not edit.  Schedules measured on AMD Radeon Graphics for R-MAT tables:
// {log2 rows, digit bits, items per thread, node method (0 sort, 1 hash)}.
#pragma once

namespace ringo {

struct TunedBucket {
  int log2_rows, digit_bits, items, node_method;
};

constexpr int NUM_TUNED = 17;
constexpr TunedBucket TUNED[NUM_TUNED > 0 ? NUM_TUNED : 1] = {
    {10, 8, 8, 0},
    {11, 8, 8, 0},
    {12, 8, 8, 0},
    {13, 8, 8, 0},
    {14, 8, 8, 0},
    {15, 8, 8, 0},
    {16, 9, 8, 0},
    {17, 9, 8, 0},
    {18, 8, 8, 0},
    {19, 8, 8, 0},
    {20, 8, 8, 0},
    {21, 8, 8, 0},
    {22, 11, 8, 1},
    {23, 10, 16, 1},
    {24, 8, 16, 1},
    {25, 8, 8, 1},
    {26, 8, 8, 1},
};

}  // namespace ringo
