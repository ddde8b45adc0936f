// Default launch schedules of FP64 plans: {log2 L, variant A, variant B,
// variant C} (variant encoding in sched.h).  Lengths not listed use variant
// 0 for every kernel.  Rows come from paper_2407_16559_amd/autotune.py run
// on an MI355X (DP5 step attempts, M = L/2); a row of -1 ends the table.
#pragma once
static const int k_sched_table[][4] = {
    {12, 2, 2, 3},  // 0.1283 -> 0.1037 ms per attempt
    {13, 0, 2, 3},  // 0.1365 -> 0.1099 ms per attempt
    {14, 0, 2, 3},  // 0.1431 -> 0.1132 ms per attempt
    {15, 0, 2, 3},  // 0.1412 -> 0.1130 ms per attempt
    {16, 0, 3, 2},  // 0.1509 -> 0.1270 ms per attempt
    {17, 0, 3, 1},  // 0.1664 -> 0.1527 ms per attempt
    {18, 0, 0, 1},  // 0.2157 -> 0.2061 ms per attempt
    {19, 0, 0, 0},  // 0.2956 -> 0.2956 ms per attempt
    {20, 0, 0, 0},  // 0.6167 -> 0.6167 ms per attempt
    {-1, 0, 0, 0},
};
