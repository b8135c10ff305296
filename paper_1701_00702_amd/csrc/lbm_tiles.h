// Tile shapes of the multi-step kernels (K = 2, 3 steps per launch through
// LDS) per storage form, shared by the kernels and host builds of the
// per-node arithmetic (the CPU replay of the step kernels in the tests).
#pragma once

#include "lbm_node.h"

namespace lbm {

constexpr int round64(int n) { return (n + 63) / 64 * 64; }

// Storage forms with a K-step kernel (K = 2, 3): two steps per launch for
// every form, three for the FP32 and 16-bit ones (an FP64 tile with a
// two-node ring leaves too few nodes per workgroup).
constexpr bool stepk_available(int st, int k) {
    const bool fp32 = st == ST_F32 || st == ST5_F32 || st == ST_F32H || st == ST5_F32H;
    const bool b16 = st == ST_F16 || st == ST_BF16 || st == ST_F16S || st == ST_BF16S;
    return k == 2 ? (fp32 || b16 || st == ST_F64 || st == ST5_F64) : (k == 3 ? (fp32 || b16) : false);
}

template <int ST>
struct Step2Tile;
// Tile shapes are build options (LBM_S2_*) for tuning; the defaults below.
#ifndef LBM_S2_F32_TW
#define LBM_S2_F32_TW 32
#define LBM_S2_F32_TH 12
#endif
#ifndef LBM_S2_F32Q5_TW
#define LBM_S2_F32Q5_TW 64
#define LBM_S2_F32Q5_TH 5
#endif
template <>
struct Step2Tile<ST_F32> {  // 27 x 4 + 4 = 112 B per slot (default 34 x 14 slots: 3 per CU)
    static constexpr int TW = LBM_S2_F32_TW, TH = LBM_S2_F32_TH, NT = round64((TW + 2) * (TH + 2));
};
template <>
struct Step2Tile<ST5_F32> {  // 19 x 4 + 4 = 80 B per slot (default 66 x 7 slots: 4 per CU)
    static constexpr int TW = LBM_S2_F32Q5_TW, TH = LBM_S2_F32Q5_TH, NT = round64((TW + 2) * (TH + 2));
};
template <>
struct Step2Tile<ST_F32H> {  // 26 x 4 + 8 + 4 = 116 B per slot, 34 x 13 slots: 3 per CU
    static constexpr int TW = 32, TH = 11, NT = 448;
};
template <>
struct Step2Tile<ST5_F32H> {  // 18 x 4 + 8 + 4 = 84 B per slot, 66 x 7 slots: 4 per CU
    static constexpr int TW = 64, TH = 5, NT = 512;
};
template <>
struct Step2Tile<ST_F16> {  // 27 x 2 + 4 = 58 B per slot, 34 x 15 slots (29 KiB)
    static constexpr int TW = 32, TH = 13, NT = 512;
};
template <>
struct Step2Tile<ST_BF16> {
    static constexpr int TW = 32, TH = 13, NT = 512;
};
template <>
struct Step2Tile<ST_F16S> {  // 6 x 4 + 24 x 2 + 4 = 76 B per slot, 34 x 15 slots (38 KiB: 4 per CU)
    static constexpr int TW = 32, TH = 13, NT = 512;
};
template <>
struct Step2Tile<ST_BF16S> : Step2Tile<ST_F16S> {};
#ifndef LBM_S2_F64_TW
#define LBM_S2_F64_TW 32
#define LBM_S2_F64_TH 5
#endif
template <>
struct Step2Tile<ST_F64> {  // 27 x 8 + 8 = 224 B per slot (default 32 x 5 with push placement: 160 slots, 37 KiB)
    static constexpr int TW = LBM_S2_F64_TW, TH = LBM_S2_F64_TH, NT = round64((TW + 2) * (TH + 2));
};
#ifndef LBM_S2_F64Q5_TW
#define LBM_S2_F64Q5_TW 32
#define LBM_S2_F64Q5_TH 8
#endif
template <>
struct Step2Tile<ST5_F64> {  // 19 x 8 + 8 = 160 B per slot (default 34 x 10 slots, 56 KiB)
    static constexpr int TW = LBM_S2_F64Q5_TW, TH = LBM_S2_F64Q5_TH, NT = round64((TW + 2) * (TH + 2));
};

// Tile shapes of the three-steps-per-launch kernel (a two-node ring; build
// options LBM_S3_* for tuning).  Measured on the 8192^2 cavity: the shape
// must leave three (D2Q9) or four (D2Q5) workgroups per CU; with two, the
// three updates and their barriers leave too little to overlap (32 x 11:
// 28.6 GLUPS against 43.7 for 32 x 9).
template <int ST>
struct Step3Tile;
#ifndef LBM_S3_F32_TW
#define LBM_S3_F32_TW 32
#define LBM_S3_F32_TH (LBM_PUSH_F32_K3 ? 8 : 9)
#endif
#ifndef LBM_S3_F32Q5_TW
#define LBM_S3_F32Q5_TW 32
#define LBM_S3_F32Q5_TH 10
#endif
template <>
struct Step3Tile<ST_F32> {  // 112 B per slot (default 32 x 8 with push placement: 34 x 10 slots, 37 KiB: 4 per CU)
    static constexpr int TW = LBM_S3_F32_TW, TH = LBM_S3_F32_TH, NT = round64((TW + 4) * (TH + 4));
};
template <>
struct Step3Tile<ST5_F32> {  // 80 B per slot (default 36 x 14 slots, 39 KiB: 4 per CU)
    static constexpr int TW = LBM_S3_F32Q5_TW, TH = LBM_S3_F32Q5_TH, NT = round64((TW + 4) * (TH + 4));
};
#ifndef LBM_S3_F16_TW
#define LBM_S3_F16_TW 32
#define LBM_S3_F16_TH 10
#endif
#ifndef LBM_S3_F16S_TW
#define LBM_S3_F16S_TW 32
#define LBM_S3_F16S_TH 10
#endif
template <>
struct Step3Tile<ST_F16> {  // 58 B per slot (default 36 x 14 slots, 29 KiB)
    static constexpr int TW = LBM_S3_F16_TW, TH = LBM_S3_F16_TH, NT = round64((TW + 4) * (TH + 4));
};
template <>
struct Step3Tile<ST_BF16> {
    static constexpr int TW = LBM_S3_F16_TW, TH = LBM_S3_F16_TH, NT = round64((TW + 4) * (TH + 4));
};
template <>
struct Step3Tile<ST_F16S> {  // 76 B per slot (default 36 x 14 slots, 38 KiB)
    static constexpr int TW = LBM_S3_F16S_TW, TH = LBM_S3_F16S_TH, NT = round64((TW + 4) * (TH + 4));
};
template <>
struct Step3Tile<ST_BF16S> : Step3Tile<ST_F16S> {};
#ifndef LBM_S3_F32H_TW
#define LBM_S3_F32H_TW 32
#define LBM_S3_F32H_TH (LBM_PUSH_F32H_K3 ? 8 : 9)
#endif
template <>
struct Step3Tile<ST_F32H> {  // 116 B per slot (push 32 x 8: 34 x 10 slots, 39 KiB, 4 per CU; pull 32 x 9: 53 KiB, 3)
    static constexpr int TW = LBM_S3_F32H_TW, TH = LBM_S3_F32H_TH, NT = round64((TW + 4) * (TH + 4));
};
template <>
struct Step3Tile<ST5_F32H> {  // 84 B per slot, 36 x 14 slots (41 KiB: 3 per CU)
    static constexpr int TW = 32, TH = 10, NT = 512;
};

template <int ST, int K>
struct StepKTile;
template <int ST>
struct StepKTile<ST, 2> : Step2Tile<ST> {};
template <int ST>
struct StepKTile<ST, 3> : Step3Tile<ST> {};

}  // namespace lbm
