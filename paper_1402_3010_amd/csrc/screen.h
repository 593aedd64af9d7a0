// Launchers of the head screen of the screened self-join (screen.hip).
#pragma once

#include "apss_internal.h"

namespace apss {

// Output tile of the screen kernel: kScreenTile rows of the packed block
// (the unit of its panels) against kScreenTileB = two such row tiles; the
// packed rows are padded to kScreenTileB.  kScreenK is the K step the
// operands are padded to (the packed head block has ld = head rounded up to
// kScreenK).
constexpr int kScreenTile = 128;
constexpr int kScreenTileB = 2 * kScreenTile;
// row tiles per side of the blocks in which the screen visits its tile list
constexpr int kScreenBlock = 8;
constexpr int kScreenK = 64;

// Screen margin coefficient: for bf16 (round to nearest even) copies of the
// head weights and float accumulation of at most head <= kScreenMaxHead
// products, |H~ - H| <= kScreenMargin * ||x_h|| ||y_h||.
constexpr int kScreenMaxHead = 8192;
constexpr float kScreenMargin = 0.0089f;
constexpr float kScreenEps = 1e-6f;

// rows with head norm >= t -> keys (~nh bits << 32 | row), count via atomic
hipError_t launch_screen_select(const RowStat* rs, int64_t n, float t, uint64_t* keys, unsigned long long* count,
                                hipStream_t s);
// sorted keys -> row ids (sid) and head norms (nh), padded to Sp with -1 / 0
hipError_t launch_screen_unpack(const uint64_t* keys, int64_t S, int64_t Sp, int32_t* sid, float* nh, hipStream_t s);
// head components (rank < head) of the selected rows -> bf16 block of Sp x ld
// (zeroed before), stored as contiguous panels of 128 rows x 32 columns,
// panel (row tile, K step) at offset (tile * ld / 32 + step) * 4096
hipError_t launch_screen_pack(const int64_t* rp, const RComp* rc, const int32_t* sid, int64_t S, int32_t head,
                              int32_t ld, uint16_t* X, hipStream_t s);

struct ScreenArgs {
  const uint16_t* X;   // Sp x ld bf16 bits in 128 x 32 panels (see launch_screen_pack)
  int32_t ld;          // multiple of kScreenK
  const float* nh;     // [Sp] head norms (rounded up), 0 for padding
  const int32_t* sid;  // [Sp] row ids
  const int32_t* tiles;  // [2 * ntiles] (I, J): rows I * kScreenTile.. against rows J * kScreenTileB..,
                         // with 2 J + 1 >= I (the tile reaches the upper triangle)
  int64_t ntiles;
  float t;
  int32_t bj;
  uint64_t* out;       // [cap] candidate keys (min id << bj | max id)
  int64_t cap;
  unsigned long long* count;
  // non-NULL: instead of testing the threshold, write every accumulated
  // head product of the tiles to dump[row * dump_ld + col] (positions in the
  // packed order); a check of the screen's error bound, not part of the join
  float* dump;
  int64_t dump_ld;
};
hipError_t launch_screen_mfma(const ScreenArgs& a, hipStream_t s);

// Verification of screen candidates: pairs that share no tail dimension
// (rank >= head) are rescored exactly (the shared rescore) and appended to
// out_key/out_sim through counters[C_MATCHES]; pairs that share one are left
// to the sparse pass.
hipError_t launch_screen_verify(const uint64_t* cand, int64_t nc, int bj, const int64_t* rp, const RComp* rc,
                                int32_t head, float t, uint64_t* out_key, float* out_sim, int64_t cap,
                                unsigned long long* counters, hipStream_t s);

}  // namespace apss
