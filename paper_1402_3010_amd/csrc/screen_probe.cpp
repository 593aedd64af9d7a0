// Check of the head screen's error bound -- a test hook, not part of the
// ABI declared in include/apss.h.
//
// apss_probe_screen_products(idx, rows, S, H, N): for the S rows `rows` of
// an index built with screen_dims > 0, packs their head components as bf16
// exactly as the screened join does and runs the screen's MFMA kernel over
// every tile pair, writing the float-accumulated head products H~[a][b]
// (a, b < S, row-major, upper triangle a <= b filled, host memory) and the
// head norms N[a] (rounded up) that the screen's margin is scaled by.  The
// test compares H~ with double-precision products to measure the margin
// |H~ - H| / (N(x) N(y)) that the screen assumes.
#include <string.h>

#include <vector>

#include "apss_internal.h"
#include "lib.h"
#include "screen.h"

using namespace apss;

extern "C" int apss_probe_screen_products(apss_index* ix, const int32_t* rows, int64_t S, float* H, float* N) {
  if (!ix || !rows || S <= 0 || !H || !N) {
    set_error("NULL or invalid argument");
    return APSS_EINVAL;
  }
  apss_index* sx = ix->screen;
  if (!sx) {
    set_error("the index was built without screen_dims");
    return APSS_EINVAL;
  }
  for (int64_t a = 0; a < S; ++a)
    if (rows[a] < 0 || rows[a] >= ix->n) {
      set_error("row %d out of range", rows[a]);
      return APSS_EINVAL;
    }
  hipStream_t s = ix->ws.stream;
  const int32_t head = sx->head_cut;
  const int32_t ld = (head + kScreenK - 1) / kScreenK * kScreenK;
  const int64_t Sp = (S + kScreenTileB - 1) / kScreenTileB * kScreenTileB;
  const int64_t T = Sp / kScreenTile, TB = Sp / kScreenTileB;
  std::vector<int32_t> tl;
  for (int64_t I = 0; I < T; ++I)
    for (int64_t J = I / 2; J < TB; ++J) {
      tl.push_back((int32_t)I);
      tl.push_back((int32_t)J);
    }
  DBuf<int32_t> sid, tiles;
  DBuf<uint16_t> X;
  DBuf<float> D;
  APSS_CHK(sid.alloc(Sp), "alloc");
  APSS_CHK(tiles.alloc((int64_t)tl.size()), "alloc");
  APSS_CHK(X.alloc(Sp * ld), "alloc");
  APSS_CHK(D.alloc(Sp * Sp), "alloc");
  APSS_CHK(hipMemcpyAsync(sid.p, rows, sizeof(int32_t) * S, hipMemcpyHostToDevice, s), "copy");
  APSS_CHK(hipMemcpyAsync(tiles.p, tl.data(), sizeof(int32_t) * tl.size(), hipMemcpyHostToDevice, s), "copy");
  APSS_CHK(fill_u32((uint32_t*)X.p, 0u, Sp * ld / 2, s), "fill");
  APSS_CHK(fill_u32((uint32_t*)D.p, 0u, Sp * Sp, s), "fill");
  APSS_CHK(launch_screen_pack(sx->rows.rp.p, sx->rows.rc.p, sid.p, S, head, ld, X.p, s), "pack");
  ScreenArgs A{};
  A.X = X.p;
  A.ld = ld;
  A.tiles = tiles.p;
  A.ntiles = (int64_t)tl.size() / 2;
  A.dump = D.p;
  A.dump_ld = Sp;
  APSS_CHK(launch_screen_mfma(A, s), "screen kernel");
  APSS_CHK(hipMemcpy2DAsync(H, sizeof(float) * S, D.p, sizeof(float) * Sp, sizeof(float) * S, S,
                            hipMemcpyDeviceToHost, s),
           "copy products");
  std::vector<RowStat> st((size_t)ix->n);
  APSS_CHK(hipMemcpyAsync(st.data(), sx->rs.p, sizeof(RowStat) * ix->n, hipMemcpyDeviceToHost, s), "copy norms");
  APSS_CHK(hipStreamSynchronize(s), "probe");
  // the head-cut index's unindexed part is the head: its norm, rounded up
  for (int64_t a = 0; a < S; ++a) N[a] = st[(size_t)rows[a]].pnrm;
  return APSS_OK;
}
