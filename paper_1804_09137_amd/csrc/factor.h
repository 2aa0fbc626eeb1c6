// Pieces shared by the translation units of the factorisation: the host
// runtime (runtime.hip), the compression of tile columns (compress_cols.hip),
// the column update (column_update.hip) and the drivers (factor.hip).
#pragma once
#include "handle.h"

#include <functional>
#include <vector>

namespace tlri {

// Issue on the side stream with the second scratch set until destroyed.
struct SideStream {
  tlr_handle_s* h;
  explicit SideStream(tlr_handle_s* hh) : h(hh) {
    swap_sets();
    h->s = h->s_side;
  }
  ~SideStream() {
    h->s = h->s_main;
    swap_sets();
  }
  void swap_sets() {
    std::swap(h->Wb, h->Wb2);
    std::swap(h->Xb, h->Xb2);
    std::swap(h->Urow, h->Urow2);
    std::swap(h->skw, h->skw2);
    std::swap(h->tw, h->tw2);
    std::swap(h->im_d, h->im2_d);
    std::swap(h->im_h, h->im2_h);
    std::swap(h->im_cap, h->im2_cap);
    std::swap(h->im_use, h->im2_use);
    std::swap(h->lm_d, h->lm2_d);
    std::swap(h->lm_h, h->lm2_h);
    std::swap(h->lm_cap, h->lm2_cap);
    std::swap(h->lm_use, h->lm2_use);
  }
};

// Issue on the diagonal-step stream until destroyed (main scratch set: only
// the diagonal factorisation's workspace is used there).
struct DiagStream {
  tlr_handle_s* h;
  explicit DiagStream(tlr_handle_s* hh) : h(hh) { h->s = h->s_diag; }
  ~DiagStream() { h->s = h->s_main; }
};

// Rank predictions for a column: final ranks and range-finder ranks.
struct RankPred {
  std::vector<int> k, r1;
  bool hist = false;   // from the same tiles of the previous factorisation (else from neighbours)
  std::vector<char> meas;   // with history: the tile was found dense by its measured rank last time
};

// A column update whose rows below the diagonal tile are left to the
// compression: those tiles still owe C_i -= W_i U^T (W: the update's left
// factor, rows from the diagonal tile on, leading dimension ldw; U: the row
// factor, nb x K).  The compression applies it inside its sketch and
// projection products instead of rewriting the whole column.  A tangent
// column also owes, per tile t, its correction C_t -= Uc_t P_t^T (Uc_t the
// primal tile's left factor in the arena, P_t = dL_jj V~_t); W then holds
// Uc_t beside the term's own columns, in columns K .. K + cr[t] of the tile's
// rows, so that one product with W^T gives both parts of the projection.
struct FoldOut {
  // in (optional): where the update builds W (wld rows apart, wcols columns
  // available) and U_row
  double* wdst = nullptr;
  int64_t wld = 0;
  int wcols = 0;
  double* udst = nullptr;
  int extra = 0;                // columns of W kept after the term's own for the correction
  // out: K > 0 when the column is folded
  const double* W = nullptr;
  int64_t ldw = 0;
  const double* U = nullptr;
  int K = 0;
  const double* zs = nullptr;   // -(Omega^T U) (and -(Omega^T Pc) after it): ld smax; null: computed here
  bool corr = false;            // the per-tile correction
  std::vector<int64_t> cu;      // Uc_t: arena offset
  std::vector<int> cr;          // Uc_t: columns (0: no correction for the tile)
  std::vector<int64_t> cp;      // P_t: first column in Pc (its Omega products: column K + cp in zs)
  const double* Pc = nullptr;   // nb x (sum cr), ld nb
};

struct ColumnJob {
  const double* src;
  int i_first, T, col;
  Family* F;
  RankPred pred;
  int64_t dense_voff;
  int g0;
  hipEvent_t wait = nullptr;   // the compression stream waits for it before reading this column
  // optional: the stream that completes this column; its first sketch is
  // launched there (after the column, ahead of that stream's later work) and
  // `wait` is recorded after it
  hipStream_t sketch_stream = nullptr;
  FoldOut fold;   // K > 0: tile t still owes C -= W[(1 + t) nb rows..] U^T
};

// One term of the left-looking sum of a TLR column update: L1(i, k) L2(j, k)^T
// with L1 from family Fi and L2 from Fj.
struct LRTerm {
  const Family* Fi;   // left factor family (tiles of rows i)
  const Family* Fj;   // right factor family (tiles of row j)
};

// runtime.hip
void rank_publish(tlr_handle_s* h, int n, bool info);
void rank_wait(tlr_handle_s* h);
void dbg_mark(tlr_handle_s* h, int id, hipStream_t st);
void dbg_host(tlr_handle_s* h, int id);
void dbg_report(tlr_handle_s* h);
int64_t apply_chunks(const HqrTask* t, int count);
const int* apply_items(tlr_handle_s* h, const HqrTask* t, int count, int* n);
hipStream_t other_stream(tlr_handle_s* h);
void prof_alone_begin(tlr_handle_s* h);
void prof_alone_end(tlr_handle_s* h);
void prof_harvest(tlr_handle_s* h);
Operand op_panels(const double* base, int64_t n, int nb, int64_t r0, int64_t c0);
GemmEpi epi_gen(const tlr_handle_s* h, int kind, int64_t grow0, int64_t gcol0);
int choose_splitk(const tlr_handle_s* h, int64_t M, int64_t N, int64_t K);
int64_t flat_tiles(tlr_handle_s* h, GemmBatch& b, int tm, int tn, const int* mh, const int* nh);
int64_t tile_take(tlr_handle_s* h, int64_t nd);
void throw_if_not_spd(tlr_handle_s* h);

// compress_cols.hip
void compress_columns(tlr_handle_s* h, std::vector<ColumnJob>& jobs, std::function<void()>* during = nullptr);
void lowrank_trsm(tlr_handle_s* h, int col, int i_first, int T, const double* vt, Family& F);

// column_update.hip
void tlr_column_update(tlr_handle_s* h, int j, int nterms, const LRTerm* terms, double* out, int epi_kind, int kb,
                       int ke, bool gen, FoldOut* fold = nullptr, hipStream_t rest_on = nullptr);

}  // namespace tlri
