// Default launch schedules of FP64 plans: {log2 L, variant A, variant B,
// variant C} (variant encoding in sched.h).  Lengths not listed use variant
// 0 for every kernel.  Rows come from paper_2407_16559_amd/autotune.py run
// on an MI355X (DP5 step attempts, M = L/2); a row of -1 ends the table.
#pragma once
static const int k_sched_table[][4] = {
    {12, 0, 2, 3},  // 0.1135 -> 0.0912 ms per attempt
    {13, 0, 2, 3},  // 0.1216 -> 0.0928 ms per attempt
    {14, 0, 2, 3},  // 0.1261 -> 0.0973 ms per attempt
    {15, 0, 2, 3},  // 0.1247 -> 0.0974 ms per attempt
    {16, 0, 3, 3},  // 0.1350 -> 0.1107 ms per attempt
    {17, 0, 3, 1},  // 0.1501 -> 0.1360 ms per attempt
    {18, 0, 0, 1},  // 0.1971 -> 0.1905 ms per attempt
    {19, 0, 0, 0},  // 0.2784 -> 0.2784 ms per attempt
    {20, 0, 0, 0},  // 0.5682 -> 0.5682 ms per attempt
    {-1, 0, 0, 0},
};
