// gp_mpnn.h - layout of the learned-proposal network (internal).
#pragma once

#include "gp_internal.h"

namespace gpk {

constexpr int kMpH = 64;                        // hidden size
constexpr int kMpF = 4;                         // input features
constexpr int kMpOffWin = 0;                    // Win[64][4]
constexpr int kMpOffBin = kMpH * kMpF;          // b_in[64]
constexpr int kMpLayer = 2 * kMpH * kMpH + kMpH;
constexpr int kMpOffL(int l) { return kMpOffBin + kMpH + l * kMpLayer; }  // Ws, Wn, b
constexpr int kMpOffWo = kMpOffL(3);            // wo[64]
constexpr int kMpOffBo = kMpOffWo + kMpH;       // bo
constexpr int kMpNParam = kMpOffBo + 1;         // 25,153
constexpr int kMpMaxN = 3072;                   // largest coarsest graph it runs on
constexpr uint32_t kMpMagic = 0x4d504e4eu;

struct MpModel {
  uint32_t magic;
  uint16_t* p;  // device, BF16 bits in blob order
};

struct MpScratch {
  uint16_t* ha;   // n x 64
  uint16_t* hb;   // n x 64
  float* inv;     // n
  float* score;   // n
  int32_t* order; // n
};

inline int next_pow2_host(int x) {
  int p = 2;
  while (p < x) p <<= 1;
  return p;
}

bool launch_mpnn_scores(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const void* model, const MpScratch& ms, hipStream_t s);
bool launch_mpnn(const LevelView& lv, const int64_t* vc, const int64_t* vg, const void* model,
                 const int64_t* tot, int gs, int npass, Ctrl* ctrl, const MpScratch& ms,
                 int8_t* out_part, hipStream_t s);

}  // namespace gpk
