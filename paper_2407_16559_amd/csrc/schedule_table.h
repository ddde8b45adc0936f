// Default launch schedules of FP64 plans: {log2 L, variant A, variant B,
// variant C} (variant encoding in sched.h).  Lengths not listed use variant
// 0 for every kernel.  Rows come from paper_2407_16559_amd/autotune.py run
// on an MI355X (DP5 step attempts, M = L/2); a row of -1 ends the table.
// Rows up to 2^17 were tuned with phase C's split workgroups (variants with
// one packed column and four waves); the longer rows, whose kernels that
// change leaves as they were, come from the tuning run before it.
#pragma once
static const int k_sched_table[][4] = {
    {12, 0, 2, 3},  // 0.1202 -> 0.0925 ms per attempt
    {13, 0, 2, 3},  // 0.1265 -> 0.0974 ms per attempt
    {14, 0, 2, 3},  // 0.1334 -> 0.1026 ms per attempt
    {15, 0, 2, 2},  // 0.1334 -> 0.0966 ms per attempt
    {16, 0, 3, 2},  // 0.1432 -> 0.1108 ms per attempt
    {17, 0, 3, 0},  // 0.1412 -> 0.1336 ms per attempt
    {18, 0, 0, 1},  // 0.1971 -> 0.1905 ms per attempt
    {19, 0, 0, 0},  // 0.2784 -> 0.2784 ms per attempt
    {20, 0, 0, 0},  // 0.5682 -> 0.5682 ms per attempt
    {-1, 0, 0, 0},
};
