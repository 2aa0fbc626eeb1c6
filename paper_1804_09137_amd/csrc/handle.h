// Private header of the library (not part of the C-ABI): the handle behind
// tlr_handle_t and the helpers shared by the factorisation's host code
// (runtime.hip, compress_cols.hip, column_update.hip, factor.hip), the C-ABI
// entry points (api.hip) and the kriging prediction (predict.hip).
#pragma once
#include "tlr.h"
#include "common.h"
#include "kernels.h"
#include "chol.h"
#include "compress.h"
#include "solve.h"
#include "grad.h"
#include "aca.h"
#include <algorithm>
#include <chrono>
#include <functional>
#include <string>
#include <thread>
#include <atomic>
#include <system_error>
#include <cstdio>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <new>
#include <string>
#include <vector>

using namespace tlrk;

namespace tlri {
constexpr int64_t kAlign = 16;
// a tangent column's correction is folded into its compression only while
// the primal column's ranks sum to at most this many columns
constexpr int kFoldRsumMax = 8192;
inline int64_t pad16(int64_t v) { return (v + kAlign - 1) / kAlign * kAlign; }
}  // namespace tlri

struct tlr_handle_s {
  tlr_opts o{};
  hipStream_t s = nullptr;        // the stream work is issued on (s_main, or s_side inside SideStream)
  hipStream_t s_main = nullptr;   // the caller's stream
  hipStream_t s_side = nullptr;   // tangent chain of the lockstep factorisation (gradient handles)
  hipStream_t s_diag = nullptr;   // gradient handles: primal diagonal steps, beside the compressions
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_px = nullptr, ev_py = nullptr;   // profiling mode 2: isolation of update groups
  hipEvent_t ev_pre = nullptr, ev_fin = nullptr; // look-ahead: side-stream pre parts done / a step's compressions done
  hipEvent_t ev_post = nullptr, ev_diag = nullptr; // a primal column complete / its diagonal step done
  hipEvent_t ev_rw = nullptr, ev_rest = nullptr;   // split update: W ready / rows below the diagonal tile done
  bool rest_pending = false;                       // ev_rest recorded, not yet waited for
  // second set of update scratch for the side stream (same capacities)
  double *Wb2 = nullptr, *Xb2 = nullptr, *Urow2 = nullptr, *skw2 = nullptr, *tw2 = nullptr;
  int device = 0;
  int64_t n = 0;
  int nb = 0, nt = 0, maxrank = 0, smax = 0;
  int gcap = 0;         // tile slots of the compression scratch
  int upd_tag = 1;      // column-update kernels of the running factorisation: 1 FP64, 2 FP32 products
  bool debug = false;   // TLR_DEBUG set: per-column compression statistics on stderr
  std::vector<hipEvent_t> dbg_ev;   // TLR_DEBUG: per-step timing marks of the three streams
  int dbg_step = -1;
  int dbg_meta_syncs = 0, dbg_meta_syncs_main = 0;   // TLR_DEBUG: staging-buffer synchronisations
  double dbg_host[8] = {0, 0, 0, 0, 0, 0, 0, 0};       // TLR_DEBUG: host time between issue points of a step
  std::chrono::steady_clock::time_point dbg_host_last{};
  double host_ms[7] = {0, 0, 0, 0, 0, 0, 0};   // TLR_DEBUG: host time in the compressions' two waits and their
                                               // callbacks, then after the second wait: bookkeeping, upload, launches
  bool pivoted_trunc = false;   // TLR_FLAG_PIVOTED_TRUNC
  bool multi = false;   // side and diagonal streams (TLR gradient handles without TLR_FLAG_SINGLE_STREAM)
  bool dense = false, grad = false, strict = false;
  int64_t vslot = 0;     // doubles per V~ staging block (nb * (maxrank + 1)): the
                         // truncating QR may produce maxrank + 1 columns before
                         // the tile is turned dense
  int64_t ntiles = 0;    // strictly-lower tiles

  const double* x = nullptr;
  const double* y = nullptr;
  double theta[3] = {0, 0, 0};
  MaternParams mp{};
  double* d_tab = nullptr;
  std::vector<double> h_tab;
  bool bound = false;
  int state = 0;  // 0 nothing; 1 compressed Sigma; 2 factor; 3 factor + tangent

  std::vector<void*> dev_allocs;
  std::vector<void*> host_allocs;
  int64_t bytes = 0;

  // factor storage
  double* Lp = nullptr;   // DENSE: lower-panel storage of L
  double* Ldp = nullptr;  // DENSE: tangent
  double* D = nullptr;    // TLR: diagonal tiles nt x (nb x nb)
  double* Dd = nullptr;   // TLR tangent diagonal tiles
  double* Dinv = nullptr; // both: inverses of the diagonal tiles (inside the arena for TLR)
  // TLR off-diagonal tiles: L_ij = U V^T with U, V (ld nb) in one arena;
  // family 0 is the factor, family 1 its tangent (gradient).  The arena
  // holds the identity block, the inverses of the diagonal tiles, then the
  // tile storage: each tile takes nb x k doubles for U and for V when its
  // rank k is known (bump allocation, reset per factorisation), so the
  // storage follows sum nb k_ij.  A tile whose rank would exceed maxrank is
  // kept dense: U = the tile itself (nb x nb), V = Dinv_j (or the identity
  // for the compressed Sigma of tlr_compress), rank = tile width.
  double* arena = nullptr;
  int64_t arena_len = 0;                 // doubles in the arena allocation
  int64_t dinv_off = 0, ident_off = 0;
  int64_t tile_off = 0, tile_cap = 0, tile_used = 0;   // tile storage: start, doubles, bump pointer
  bool tile_auto = true;                 // opts.arena_bytes == 0: grow the storage when a factor needs more
  bool tile_overflow = false;            // the last failure was the tile storage running out
  int arena_grows = 0;
  int splitk_count = 0;                  // split-K GEMM launches of the running factorisation
  int qr_class[3] = {0, 0, 0};           // truncation QRs by size class (registers, + LDS, global)
  struct Family {
    std::vector<int> rk;                 // nt*nt (i * nt + j)
    std::vector<int> r1;                 // range-finder ranks (sketch width prediction)
    std::vector<int> r1_prev, rk_prev;   // the previous factorisation's ranks, if hist
    bool hist = false;
    int done_kind = 0;                   // what the last finished pass computed: 1 factor, 2 compression of Sigma
    std::vector<int64_t> uoff, voff;     // arena offsets of U_ij, V_ij
    std::vector<char> isdense;
    std::vector<char> dense_meas, dense_meas_prev;   // dense by a measured rank (not decided early), this / last pass
    int* rk_d = nullptr;
    int64_t* uoff_d = nullptr;
    int64_t* voff_d = nullptr;
  } fam[2];

  // scratch
  double* colbase = nullptr;  // the column buffers, one allocation (compressions address tiles from here)
  double* col = nullptr;      // n x nb, ld n
  double* cold = nullptr;     // tangent column
  double* col2 = nullptr;     // gradient handles: second primal and tangent columns, so that the
  double* cold2 = nullptr;    //   next step's update can run while a column is compressed
  double* omega = nullptr; // nb x smax
  double* Ybuf = nullptr;  // nt blocks of nb x smax (ld nb): sketches, then small-QR workspace
  double* Q1 = nullptr;    // nt blocks of nb x smax (ld nb): range bases
  double* Bt = nullptr;    // nt x (nb x smax)
  double* Vtmp = nullptr;  // gcap x vslot: V~ of the tiles being compressed
  double* Ptmp = nullptr;  // nt x nb x nb (gradient: dL_jj V_ij products)
  int64_t ptmp_cap = 0;
  double* Zb = nullptr;    // nt x (smax x maxrank)
  double* Wb = nullptr;
  int64_t w_cap = 0;
  double* Xb = nullptr;
  int64_t x_cap = 0;
  double* Urow = nullptr;
  int64_t urow_cap = 0;
  double* skw = nullptr;
  int64_t sk_cap = 0;
  double* tw = nullptr;    // 64 * nb (+ nb * nb tangent scratch)
  double* vec = nullptr;   // 4 vectors of n
  double* scal = nullptr;  // device scalars: [0, nt) log-diag, [nt, 2nt) tangent traces, ...
  double* h_scal = nullptr;
  unsigned long long* info_d = nullptr;
  unsigned long long* h_info = nullptr;

  // per-launch metadata, bump-allocated per column
  int* im_d = nullptr;
  int* im_h = nullptr;
  int64_t im_cap = 0, im_use = 0;
  int64_t* lm_d = nullptr;
  int64_t* lm_h = nullptr;
  int64_t lm_cap = 0, lm_use = 0;
  // the side stream's own staging set (swapped in with the side stream)
  int* im2_d = nullptr;
  int* im2_h = nullptr;
  int64_t im2_cap = 0, im2_use = 0;
  int64_t* lm2_d = nullptr;
  int64_t* lm2_h = nullptr;
  int64_t lm2_cap = 0, lm2_use = 0;
  QrcpTask* tk_d = nullptr;
  QrcpTask* tk_h = nullptr;
  int tk_cap = 0;
  HqrTask* hq_d = nullptr;  // 6 x gcap: one region per launch between synchronisations
  HqrTask* hq_h = nullptr;
  double* Tw = nullptr;     // nt x tw_stride compact-WY factors
  int64_t tw_stride = 0;
  double* Tr = nullptr;     // gcap x tr_stride compact-WY factors of the truncation QR's reflectors
  int64_t tr_stride = 0;
  double* Tau = nullptr;    // gcap x kRegQrBig reflector scalars of the truncation QR
  double* zst = nullptr;    // smax x maxrank: -(Omega^T U) of a folded column update
  double* lrtws = nullptr;  // nt x kLrMaxRank: the low-rank apply's t = B^T v per tile
  double* gbuf = nullptr;   // -(W_i^T Q1_i) of a folded column's tiles, gbuf_cap doubles
  int64_t gbuf_cap = 0;
  // the W of folded column updates: the primal column's (wf_ld rows apart,
  // wf_pcols columns) then the tangent column's (wf_tcols columns), one
  // leading dimension so that one launch takes the projections' W^T Q1
  double* Wf = nullptr;
  int64_t wf_cap = 0, wf_ld = 0;
  int wf_pcols = 0, wf_tcols = 0;
  double* zst2 = nullptr;   // smax x zst2_cols: -(Omega^T [U P]) of a folded tangent column
  int zst2_cols = 0;
  AcaTask* aca_d = nullptr;  // gcap ACA task records (tlr_compress with TLR_FLAG_ACA)
  AcaTask* aca_h = nullptr;
  int* qr_d = nullptr;  // 2 * gcap: ranks, flags
  int* qr_h = nullptr;  // fine-grained host copy (rank_publish), device address qr_hd
  int* qr_hd = nullptr;
  unsigned long long* h_info_d = nullptr;   // device address of h_info (fine-grained)
  unsigned* pub_seq_h = nullptr;            // last publish sequence number written by the device
  unsigned* pub_seq_d = nullptr;
  unsigned pub_seq = 0;                     // last one issued
  // FP32-product check (TLR_PREC_FP32_UPDATES handles): per diagonal tile j,
  // chk[2j] = ||A_jj - D~_jj||_F^2 (the update that reached the tile) and
  // chk[2j+1] = ||D_jj^{-1}||_F^2; chk_scr is one nb x nb scratch tile
  double* chk_d = nullptr;
  double* chk_h = nullptr;
  double* chk_scr = nullptr;

  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // per-kernel-class event timing (tlr_profile)
  int prof = 0;         // 0 off, 1 event pairs per launch group, 2 the same with update groups run alone
  std::vector<hipEvent_t> evpool;
  size_t ev_used = 0;
  struct Pending { int cls; size_t e0, e1; double flops, bytes; };
  std::vector<Pending> pend;
  tlr_kstat kst[TLR_K_COUNT]{};
  tlr_info info{};
  int bad_i = -1, bad_j = -1;
};

namespace tlri {
using namespace tlrk;

// Internal failure: thrown by the helpers, turned into the status code at the
// C-ABI by guarded().
struct Fail {
  tlr_status st;
};



#define NOMEM(what) nomem(what, __FILE__, __LINE__)

#define HIPCHK(x)                                    \
  do {                                               \
    hipError_t e_ = (x);                             \
    if (e_ != hipSuccess) hip_fail(e_, #x, __FILE__, __LINE__); \
  } while (0)

template <class T>
T* dalloc(tlr_handle_s* h, int64_t count) {
  if (count <= 0) count = 1;
  void* p = nullptr;
  if (hipMalloc(&p, (size_t)count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{TLR_ENOMEM};
  }
  h->dev_allocs.push_back(p);
  h->bytes += count * (int64_t)sizeof(T);
  return (T*)p;
}

template <class T>
T* halloc(tlr_handle_s* h, int64_t count, unsigned flags = hipHostMallocDefault) {
  if (count <= 0) count = 1;
  void* p = nullptr;
  if (hipHostMalloc(&p, (size_t)count * sizeof(T), flags) != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{TLR_ENOMEM};
  }
  h->host_allocs.push_back(p);
  return (T*)p;
}
// Fine-grained (coherent) host memory that kernels write and the host polls;
// *dev receives the device address of the same bytes.
template <class T>
T* halloc_coherent(tlr_handle_s* h, int64_t count, T** dev) {
  T* p = halloc<T>(h, count, hipHostMallocCoherent | hipHostMallocMapped);
  void* d = nullptr;
  if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
    (void)hipGetLastError();
    throw Fail{TLR_ENOMEM};
  }
  *dev = (T*)d;
  return p;
}

extern thread_local char g_last_error[256];
[[noreturn]] void hip_fail(hipError_t e, const char* what, const char* file, int line);
[[noreturn]] void nomem(const char* what, const char* file, int line);

inline int tile_rows(const tlr_handle_s* h, int i) {
  return (i == h->nt - 1) ? (int)(h->n - (int64_t)i * h->nb) : h->nb;
}
inline double* dinv_tile(tlr_handle_s* h, int j) { return h->Dinv + (int64_t)j * h->nb * h->nb; }
inline double* diag_tile(tlr_handle_s* h, int j) { return h->D + (int64_t)j * h->nb * h->nb; }
using Family = tlr_handle_s::Family;
inline size_t tid_of(const tlr_handle_s* h, int i, int j) { return (size_t)i * h->nt + j; }

// ---- drivers (factor.hip, runtime.hip) used by the entry points ----
void sync(tlr_handle_s* h);
void free_all(tlr_handle_s* h);
float elapsed(hipEvent_t a, hipEvent_t b);
void reset_info(tlr_handle_s* h);
void rank_stats(tlr_handle_s* h);
tlr_status factor_checked(tlr_handle_s* h, bool tangent, int64_t* info);
bool fp32_check_fails(tlr_handle_s* h, double ll);
void solve_forward(tlr_handle_s* h, const double* z, double* logdet, double* quad);
void solve_backward(tlr_handle_s* h);
void compress_sigma(tlr_handle_s* h);
void compress_sigma_aca(tlr_handle_s* h);
void arena_alloc(tlr_handle_s* h, int64_t cap);
void arena_grow(tlr_handle_s* h);
void arena_ensure(tlr_handle_s* h);
void family_reset(tlr_handle_s* h, Family& F, int kind);
void drop_history(tlr_handle_s* h);
void family_upload(tlr_handle_s* h, Family& F);
int lr_kmax(const tlr_handle_s* h, int j, bool col);
double* panel(tlr_handle_s* h, double* base, int j);
// per-launch metadata staging and per-class event timing
int* im_take(tlr_handle_s* h, int64_t cnt, int** dptr);
int64_t* lm_take(tlr_handle_s* h, int64_t cnt, int64_t** dptr);
void im_push(tlr_handle_s* h, const int* hp, int* dp, int64_t cnt);
void lm_push(tlr_handle_s* h, const int64_t* hp, int64_t* dp, int64_t cnt);
void meta_reset(tlr_handle_s* h);
void meta_reserve(tlr_handle_s* h, int64_t ints, int64_t longs);
size_t prof_mark(tlr_handle_s* h);
void prof_add(tlr_handle_s* h, int cls, size_t e0, double flops, double bytes);
void prof_reset_pool(tlr_handle_s* h);
// GEMM through the handle's stream (optional split-K, flat tile lists)
Operand op_contig(const double* base, int64_t ld, int64_t r0 = 0, int64_t c0 = 0);
Operand op_contigT(const double* base, int64_t ld, int64_t r0 = 0, int64_t c0 = 0);
GemmEpi epi_linear(double alpha, double beta);
void gemm(tlr_handle_s* h, int64_t M, int64_t N, int nseg, const GemmSeg* segs, double* C, int64_t ldc,
          const GemmEpi& ep, const GemmBatch* b = nullptr, bool allow_split = false, int tm = 0, int tn = 0,
          const int* mh = nullptr, const int* nh = nullptr, int tag = 0);

// Runs f, turning a Fail into its status (the handle's streams are drained
// first unless the failure was an allocation).
template <class F>
tlr_status guarded(tlr_handle_s* h, F&& f) {
  try {
    return f();
  } catch (const Fail& e) {
    if (h && e.st == TLR_ERANK) {
      h->info.bad_tile_i = h->bad_i;
      h->info.bad_tile_j = h->bad_j;
    }
    if (h && e.st != TLR_ENOMEM) {
      (void)hipStreamSynchronize(h->s_main);
      if (h->s_side) (void)hipStreamSynchronize(h->s_side);
      if (h->s_diag) (void)hipStreamSynchronize(h->s_diag);
    }
    return e.st;
  } catch (const std::bad_alloc&) {
    return TLR_ENOMEM;
  }
}

}  // namespace tlri
