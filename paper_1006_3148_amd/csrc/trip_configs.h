// Tile shapes the trip kernel is compiled for.
#pragma once

// Compiled tile shapes: R rows per wave x W waves (tile = 64 x R*W columns)
// for T = 1..8.  Configurations whose per-stage register state spills are
// still compiled; the host only picks shapes that trip_config_supported lists.
#define JACOBI_TRIP_CFGS(X) \
    X(1, 4, 16) X(2, 4, 16)                                                   \
    X(1, 4, 8) X(2, 4, 8) X(3, 4, 8) X(4, 4, 8) X(5, 4, 8) X(6, 4, 8)          \
    X(1, 2, 16) X(2, 2, 16) X(3, 2, 16) X(4, 2, 16) X(5, 2, 16) X(6, 2, 16)    \
    X(7, 2, 16) X(8, 2, 16) X(7, 4, 8) X(8, 4, 8)                             \
    X(2, 4, 12) X(3, 3, 12) X(4, 3, 12) X(4, 4, 12) X(5, 3, 12) X(5, 4, 12)   \
    X(6, 3, 12) X(3, 4, 12)

// Tile shapes of the 27-point update (FP64, A/B): six FP64 values of
// k-streaming state per stage and cell instead of two, so fewer stages fit in
// the registers of a 512-thread workgroup.
#define JACOBI_S27_CFGS(X) \
    X(1, 4, 8) X(2, 4, 8) X(2, 3, 12) X(2, 2, 16) X(3, 3, 8) X(3, 4, 8) X(4, 3, 8)
