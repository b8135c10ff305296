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
#define LBM_S3_F32H_TH (LBM_PUSH_F32H_K3 ? 10 : 9)
#endif
template <>
struct Step3Tile<ST_F32H> {  // 116 B per slot (push 32 x 10: 34 x 12 slots, 46 KiB, 3 per CU, 45.7 GLUPS
                             // on the 8192^2 cavity against 45.1 for 32 x 8 with 4 per CU; pull 32 x 9: 53 KiB, 3)
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

// Tile shapes chosen at run time (lbm_launch_config.tile_shape): 0 is the
// default above; 1 is about twice as wide and half as tall, 2 about half as
// wide and twice as tall, each within 64 KiB of LDS, 1024 threads and the
// band rule (TH + 2K <= LBM_MIN_BAND_ROWS).  The autotuner times them: a
// cavity whose width leaves a narrow last tile in one shape fits another.
constexpr int kTileShapes = 3;
struct TileDims {
    int tw, th;
};
constexpr TileDims alt_dims(int st, int k, int i) {
    if (k == 3) {
        if (st == ST_F32 || st == ST_F32H) return i == 1 ? TileDims{64, 4} : TileDims{16, 16};
        return i == 1 ? TileDims{64, 5} : TileDims{16, 20};  // D2Q5 FP32 forms, 16-bit forms
    }
    switch (st) {
        case ST_F32: return i == 1 ? TileDims{64, 6} : TileDims{16, 24};
        case ST_F32H: return i == 1 ? TileDims{64, 5} : TileDims{16, 22};
        case ST5_F32:
        case ST5_F32H: return i == 1 ? TileDims{32, 10} : TileDims{128, 3};
        case ST_F64: return i == 1 ? TileDims{64, 3} : TileDims{16, 10};
        case ST5_F64: return i == 1 ? TileDims{64, 4} : TileDims{16, 16};
        default: return i == 1 ? TileDims{64, 6} : TileDims{16, 26};  // 16-bit forms
    }
}
template <int ST, int K, int I>
struct StepKTileI {
    static constexpr TileDims d = alt_dims(ST, K, I);
    static constexpr int TW = d.tw, TH = d.th, NT = round64((TW + 2 * (K - 1)) * (TH + 2 * (K - 1)));
};
template <int ST, int K>
struct StepKTileI<ST, K, 0> : StepKTile<ST, K> {};

// Width and height of tile shape i of the K-step kernel of storage st.
template <int ST, int K>
constexpr TileDims dims_of(int i) {
    return i == 0 ? TileDims{StepKTile<ST, K>::TW, StepKTile<ST, K>::TH} : alt_dims(ST, K, i);
}

}  // namespace lbm
