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

// phi(x) = (bitlen(x) - 1) + (the 8 bits after the leading one) / 256, and 0
// for x <= 0.  Computed on 32-bit words: the leading word is normalised so
// that its top bit is the leading one, then the next 8 bits are read off.
// No 64-bit shift by a variable amount appears, so the float conversions are
// 32-bit too (see the shift check in the build script).
__device__ __forceinline__ float mp_phi(int64_t x) {
  if (x <= 0) return 0.0f;
  const uint32_t hi = (uint32_t)((uint64_t)x >> 32), lo = (uint32_t)(uint64_t)x;
  const uint32_t t = hi ? hi : lo, tl = hi ? lo : 0u;
  const int c = __clz((int)t);
  const uint32_t top = c ? ((t << c) | (tl >> (32 - c))) : t;
  const uint32_t e = (hi ? 63u : 31u) - (uint32_t)c;
  return (float)e + (float)((top >> 23) & 0xffu) * (1.0f / 256.0f);
}

inline int next_pow2_host(int x) {
  int p = 2;
  while (p < x) p <<= 1;
  return p;
}

bool launch_mpnn_scores(const LevelView& lv, const int64_t* vc, const int64_t* vg,
                        const void* model, const MpScratch& ms, hipStream_t s);
// the refined learned proposal of the coarsest graph: assignment to lp_out
// (int8[n]), part weights to lpw_out (int64[2], device)
bool launch_mpnn(const LevelView& lv, const int64_t* vc, const int64_t* vg, const void* model,
                 int gs, int npass, const Ctrl* ctrl, const MpScratch& ms, int8_t* lp_out,
                 int64_t* lpw_out, hipStream_t s);

}  // namespace gpk
