// gp_internal.h - layouts shared by the host driver and the gfx950 kernels.
//
// Vertex ids are int32, weights, gains, cut and loads int64.  A level of the
// multilevel hierarchy is a symmetric CSR graph with rows sorted by
// neighbour id and two cost columns (cpu, gpu) kept as separate arrays, so
// the balance column is one contiguous int64 stream.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gpk {

constexpr int kBlock = 256;       // threads per block of the level kernels
constexpr int kTileV = 1024;      // vertices per tile of the ordered-scan kernels
constexpr int kMatchSegMax = 4096;  // blocks (list segments) of a matching round
constexpr int kContractSegMax = 16384;  // blocks (row segments) of the short-row kernel
constexpr int kPartials = 5 * 8192;  // int64 scratch of the reductions and the segment lists
constexpr int kTileC = 64;        // coarse rows per tile of the row-sort kernel
constexpr int kWaveCap = 512;     // longest candidate row sorted in LDS by one wave
constexpr int kRowBlockCap = 2048;  // longest candidate row sorted in LDS by one block (contraction)
constexpr int kSortCap = 4096;    // longest candidate row sorted in LDS by one block
constexpr int kWin = 4096;        // id window of the dense long-row merge
constexpr int kLongCap = 4096;    // longest candidate row one wave can sort with packed keys
// longest row given to one wave by the single-graph path (longer rows take a
// block each: four waves per row beat one beyond it)
constexpr int kLongWave = 2048;
constexpr int kPackIdBits = 12;   // position bits of a packed key: kLongCap = 2^12
constexpr int32_t kPackMaxNc = (1 << 19) - 1;  // coarse ids below this fit a packed key
constexpr int kMaxLevels = 48;
constexpr int kMaxRounds = 64;
constexpr int kInitBlock = 64;    // one wave per greedy-growing trial

// candidate of a refinement pass: admission order is gain desc, id asc
// b: weight the move adds to the destination side; bs: weight it takes from
// the source side (equal unless the two sides are measured in different
// columns: time balance)
struct Cand {
  int64_t gain;
  int64_t b;
  int64_t bs;
  int32_t v;
  int32_t pad;
};

enum : int32_t { kAdmitNone = 0, kAdmitAll = 1, kAdmitThr = 2 };

// one refinement state (the whole-graph one, or one per initial trial)
struct RefCtl {
  int64_t pw[2];
  int64_t maxw[2];
  int32_t pass, z, done, npass;   // npass = P
  int32_t mode, s;                // mode 0 improvement, 1 rebalance; s = side that moves
  int32_t admit, idbits;
  uint64_t thr_hi, thr_lo;        // admit iff key >= thr (128-bit key)
  int64_t gmin;                   // gain offset of the key
  // per-pass accumulators, cleared after each pass
  int64_t ext_sum;                // sum over vertices of ext = 2 x cut at pass start
  int64_t cand_b;
  int64_t gmin_acc, gmax_acc;
  uint32_t ncand;
  uint32_t pad0;
  int64_t moved_b, moved_n, moved_bs;
  // totals
  int64_t total_moves;
  int64_t last_cut;
  uint32_t ctr_gain, ctr_apply;   // last-block counters
  // the pass just finished (kept for the neighbour updates that follow it)
  uint32_t last_ncand;            // candidates listed
  int32_t last_d;                 // side the moved vertices joined
  int64_t last_moved_n;           // vertices moved
};

struct Ctrl {
  RefCtl ref;
  int64_t tgt[2];
  int64_t cap;            // matching weight cap
  int64_t maxb;           // largest balance weight on the current level
  int32_t made[kMaxRounds];
  // contraction
  int32_t nc, nnz_c, nlong, nhuge;  // nhuge: rows sorted by one block each
  int64_t ubtot;
  int64_t long_in, long_out;  // candidates read and entries written by the long-row kernel
  int64_t huge_in, huge_out;  // the same for the rows of one block each
  int64_t short_in, short_out;  // the same for the rows of <= 32 candidates
  int64_t deferred;            // rows the short-row kernel left to the row kernel
  int64_t maxb_next;
  uint32_t ctr_count, ctr_long, ctr_stats, ctr_init;
  int32_t niso;           // unmatched vertices without neighbours
  uint32_t ctr_iso;
  int32_t lvl_pass[kMaxLevels + 1];  // refinement passes run on each level
  int32_t used_learned;              // the learned proposal replaced the plain one
  int32_t pad2;
  int64_t lpw[2];                    // part weights of the refined learned proposal
  // result of the final statistics kernel
  int64_t res_ext, res_load[2], res_time[2];
  int64_t res_vol;        // communication volume (volume objective)
  // validation
  uint32_t verr;          // bit flags
  uint32_t vunsorted;
  uint64_t vsum_w, vsum_c, vsum_g;
  int64_t vmax_c, vmax_g;
};

// validation flag bits
enum : uint32_t {
  kVInval = 1u, kVRange = 2u, kVSelf = 4u, kVDup = 8u, kVAsym = 16u, kVOverflow = 32u
};

// device view of one level.  Row u is adj / w [xadj[u], xend[u]).  A level
// built by the single-graph contraction keeps each row where its upper bound
// put it, so rows may have gaps between them; a compact level (the input
// graph, the coarsest level, every level of the batched path) has
// xend = xadj + 1.  nnz counts the entries, not the span.
struct LevelView {
  int32_t n, nnz;
  const int32_t* xadj;
  const int32_t* adj;
  const int64_t* w;
  const int64_t* b;     // balance column
  const int32_t* xend;
};

}  // namespace gpk
