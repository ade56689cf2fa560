// FFT lengths with a compiled kernel set, and the radix of each Stockham
// stage (non-increasing; 1 = no stage). Shared by the host planner, which
// pads every grid dimension to the smallest listed length >= 2 N_d - 1, and
// by the device passes, which are instantiated once per entry.
#pragma once

#define AIM_FOR_EACH_FFT_PLAN(X) \
  X(5, 5, 1, 1)                  \
  X(6, 6, 1, 1)                  \
  X(8, 8, 1, 1)                  \
  X(9, 9, 1, 1)                  \
  X(10, 10, 1, 1)                \
  X(12, 12, 1, 1)                \
  X(14, 14, 1, 1)                \
  X(16, 16, 1, 1)                \
  X(18, 18, 1, 1)                \
  X(21, 7, 3, 1)                 \
  X(24, 6, 4, 1)                 \
  X(27, 9, 3, 1)                 \
  X(32, 8, 4, 1)                 \
  X(36, 6, 6, 1)                 \
  X(42, 7, 6, 1)                 \
  X(48, 8, 6, 1)                 \
  X(54, 9, 6, 1)                 \
  X(63, 9, 7, 1)                 \
  X(72, 9, 8, 1)                 \
  X(81, 9, 9, 1)                 \
  X(96, 12, 8, 1)                \
  X(108, 12, 9, 1)               \
  X(126, 14, 9, 1)               \
  X(144, 12, 12, 1)              \
  X(162, 18, 9, 1)               \
  X(192, 16, 12, 1)              \
  X(216, 18, 12, 1)              \
  X(243, 9, 9, 3)                \
  X(288, 18, 16, 1)              \
  X(324, 18, 18, 1)              \
  X(384, 16, 8, 3)               \
  X(432, 12, 6, 6)               \
  X(486, 18, 9, 3)               \
  X(576, 12, 8, 6)               \
  X(648, 18, 6, 6)               \
  X(768, 16, 8, 6)               \
  X(864, 12, 9, 8)               \
  X(972, 18, 9, 6)               \
  X(1152, 16, 9, 8)              \
  X(1296, 18, 9, 8)              \
  X(1536, 16, 12, 8)             \
  X(1728, 16, 12, 9)             \
  X(2048, 16, 16, 8)             \
  X(2304, 16, 16, 9)             \
  X(2592, 18, 16, 9)             \
  X(3072, 16, 16, 12)            \
  X(3456, 18, 16, 12)
