// Default launch schedules of FP64 plans: {log2 L, variant A, variant B,
// variant C} (variant encoding in sched.h).  Lengths not listed use variant
// 0 for every kernel.  Rows come from paper_2407_16559_amd/autotune.py run
// on an MI355X (DP5 step attempts, M = L/2); a row of -1 ends the table.
#pragma once
static const int k_sched_table[][4] = {
    {12, 2, 2, 3},  // 0.1325 -> 0.1024 ms per attempt
    {13, 2, 2, 2},  // 0.1395 -> 0.1096 ms per attempt
    {14, 2, 2, 2},  // 0.1454 -> 0.1122 ms per attempt
    {15, 0, 2, 2},  // 0.1457 -> 0.1142 ms per attempt
    {16, 0, 3, 2},  // 0.1517 -> 0.1226 ms per attempt
    {17, 0, 3, 1},  // 0.1701 -> 0.1526 ms per attempt
    {18, 0, 0, 1},  // 0.2084 -> 0.2017 ms per attempt
    {19, 0, 0, 0},  // 0.3096 -> 0.3096 ms per attempt
    {20, 0, 0, 0},  // 0.6263 -> 0.6263 ms per attempt
    {-1, 0, 0, 0},
};
