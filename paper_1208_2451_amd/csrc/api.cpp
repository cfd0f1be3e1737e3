// Host driver and C ABI of the gfx950 LU_PRRP / CALU_PRRP library.
//
// prrp_factor runs Algorithm "LU_PRRP factorization" (Section 2.1) one panel
// at a time on one stream:
//   srrqr  -- strong RRQR of the panel transpose (pivot rows, M = R11^-1 R12)
//   gepp   -- transposition plan, GEPP of the b x b block, Pi11 L11
//   moves  -- the row interchanges applied to the columns outside the panel
//   trsm   -- U12 = L11^-1 A12
//   gemm   -- L21 = M^T (Pi11 L11), A22 -= L21 U12
// calu_prrp_factor replaces the srrqr step by a tournament (Section 3.1):
// strong RRQR of every row tile, then of stacked candidate pairs up a binary
// tree (or along a chain), and finally the QR with the winners as pivots.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>
#include <vector>
#include <cstdlib>
#include <mutex>

#include "common.h"
#include "kernels.h"
#include "prrp.h"

using namespace prrp;

namespace {

constexpr int kRoundsMax = kMaxB + kMaxExchange + 2;
constexpr int kRowsPerWgMax = 128;   // 32 row groups x 4 rows per thread
constexpr int kRowsOneWg = 256;      // one 1024-thread workgroup (at most 64 columns)

inline uint64_t tau_bits(double tau) {
  uint64_t u;
  std::memcpy(&u, &tau, sizeof u);
  return u >> kDropBits;
}

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

int device_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
      cus = 256;
  }
  return cus;
}

struct Tiles {
  std::vector<int> start, len;
};

// Top-down tiles of tile_rows rows; a last remainder of <= b rows joins the
// previous tile.
Tiles tile_bounds(int64_t m, int64_t tile_rows, int b) {
  Tiles t;
  for (int64_t s = 0; s < m; s += tile_rows) {
    t.start.push_back((int)s);
    t.len.push_back((int)std::min<int64_t>(tile_rows, m - s));
  }
  if (t.start.size() > 1 && t.len.back() <= b) {
    t.len[t.len.size() - 2] += t.len.back();
    t.start.pop_back();
    t.len.pop_back();
  }
  return t;
}

// Workgroups per tile.  Each pivot step costs one device-scope round trip
// whose latency grows with the number of workgroups polled (~1.8 us at 64,
// ~3.3 us at 256 on MI355X), while fewer workgroups mean more rows each (at
// most 128, the register budget).  Default: at most 64 rows per workgroup,
// at most PRRP_PANEL_WGS (default 64, within the CUs the look-ahead keeps
// free of the trailing update) workgroups; none left without rows.
int panel_wg_cap() {
  static int cap = 0;
  if (cap == 0) {
    const char* e = getenv("PRRP_PANEL_WGS");
    cap = e ? atoi(e) : 64;
    if (cap < 1) cap = 1;
    if (cap > 256) cap = 256;
  }
  return cap;
}

// A tile of at most 128 rows, or of at most 256 rows and 64 columns, is held
// by one workgroup (PRRP_ONE_WG=0 splits it as any other tile): its steps
// then wait on barriers only.
bool one_wg_tiles() {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("PRRP_ONE_WG");
    on = (e && atoi(e) == 0) ? 0 : 1;
  }
  return on == 1;
}

// PRRP_INTERLEAVE=0 keeps each tile's workgroups in consecutive blocks.
bool interleave_tiles() {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("PRRP_INTERLEAVE");
    on = (e && atoi(e) == 0) ? 0 : 1;
  }
  return on == 1;
}

// `target` rows per workgroup (64 or 128); the workspace is always sized for
// the default 64, which gives the most workgroups.
int groups_for_rows(int64_t rows, int cap, int target, int bw) {
  if (one_wg_tiles() && (rows <= kRowsPerWgMax || (rows <= kRowsOneWg && bw <= 64))) return 1;
  cap = std::min(cap, panel_wg_cap());
  int G = (int)std::min<int64_t>(cap, (rows + target - 1) / target);
  if (G < 1) G = 1;
  while ((rows + G - 1) / G > kRowsPerWgMax) ++G;
  const int64_t rpw = (rows + G - 1) / G;
  return (int)std::max<int64_t>(1, (rows + rpw - 1) / rpw);
}

// Compute units that one strong-RRQR tile of G workgroups (bw columns, rpw
// rows each) occupies when all of them are resident -- or `total` workgroups
// of such tiles, when given -- or -1 if the occupancy query fails.  Every
// workgroup of a tile waits on the others, so the tile must fit at once.
int64_t tile_cus(int G, int bw, int rpw, int bpc_given = 0, int64_t total = 0) {
  const int64_t wgs = total > 0 ? total : G;
  if (bpc_given > 0) return (wgs + bpc_given - 1) / bpc_given;
  static std::mutex mu;
  static std::vector<std::pair<int64_t, int>> cache;   // ((bw, rpw, G <= 16), blocks)
  const int64_t key = ((int64_t)bw << 32) | ((int64_t)(G <= 16) << 31) | (uint32_t)rpw;
  int bpc = 0;
  {
    std::lock_guard<std::mutex> g(mu);
    for (auto& kv : cache) if (kv.first == key) bpc = kv.second;
    if (bpc == 0) {
      if (srrqr_blocks_per_cu(bw, rpw, G, &bpc) != hipSuccess || bpc < 1) return -1;
      cache.push_back({key, bpc});
    }
  }
  return (wgs + bpc - 1) / bpc;
}

struct Layout {
  size_t slots_set_words = 0;     // words per slot set
  size_t off_slots = 0, off_rounds = 0, off_abort = 0, off_sel = 0, off_lists = 0;
  size_t off_y = 0, off_pl = 0, off_p11 = 0, off_moves = 0, off_lsel = 0;
  size_t off_panel = 0, off_srcmap = 0, panel_stride = 0, off_winv = 0;
  size_t y_stride = 0, sel_stride = 0;   // the two panels' Y and sel buffers
  size_t total = 0;
  int max_members = 0;            // sum over groups of workgroups in any launch
  int max_groups = 0;
};

Layout make_layout(int64_t n, int b, int method, int64_t tile_rows) {
  Layout L;
  const int cap = std::min(256, device_cus());
  int members = groups_for_rows(n, cap, 64, b);
  int groups = 1;
  if (method == 1) {
    const int64_t ntiles = (n + tile_rows - 1) / tile_rows;
    const int Gl = groups_for_rows(std::min<int64_t>(tile_rows + b, n), cap, 64, b);
    members = std::max<int64_t>(members, ntiles * Gl);
    members = std::max<int64_t>(members, ((ntiles + 1) / 2) * groups_for_rows(2 * b, cap, 64, b));
    members = std::max<int>(members, groups_for_rows(tile_rows + b + b, cap, 64, b));
    groups = (int)std::max<int64_t>(1, ntiles);
  }
  L.max_members = members;
  L.max_groups = groups;
  L.slots_set_words = (size_t)members * kRoundsMax * kPostW;
  size_t off = 0;
  L.off_slots = off;  off += align_up(2 * L.slots_set_words * 8, 256);
  L.off_rounds = off; off += align_up(2 * (size_t)groups * 4 + 16, 256);
  L.off_abort = off;  off += 256;
  L.off_sel = off;    off += align_up((size_t)2 * groups * kMaxB * 4, 256);   // two panels
  L.off_lsel = off;   off += align_up((size_t)2 * groups * kMaxB * 4, 256);
  L.off_lists = off;  off += align_up((size_t)groups * (2 * kMaxB + (size_t)tile_rows + 64) * 4 + 64, 256);
  L.off_y = off;      off += 2 * align_up((size_t)n * b * 8, 256);         // two panels
  L.y_stride = align_up((size_t)n * b * 8, 256);
  L.sel_stride = (size_t)groups * kMaxB;
  L.off_pl = off;     off += align_up((size_t)b * b * 8, 256);
  L.off_p11 = off;    off += align_up((size_t)kMaxB * 4, 256);
  L.off_moves = off;  off += 2 * align_up((size_t)(4 * kMaxB + 4) * 4, 256);
  // the next panel's columns after the near update (two panels, n x b each)
  L.panel_stride = align_up((size_t)n * b * 8, 256);
  L.off_panel = off;  off += 2 * L.panel_stride;
  L.off_srcmap = off; off += align_up((size_t)n * 4, 256);
  L.off_winv = off;   off += align_up((size_t)b * b * 8, 256);   // CALU_PRRP root: A11^-1
  L.total = off;
  return L;
}

inline int herr(hipError_t e) { return e == hipSuccess ? 0 : -1000 - (int)e; }

// ------------------------------------------------ look-ahead side stream
// The far part of each Schur update runs on a side stream whose CU mask
// leaves PRRP_RESERVE_CUS (default 96, 12 per XCD) CUs free, so that the
// next panel's latency-bound kernels (strong RRQR, GEPP) always find free CUs
// and run concurrently with it.  Measured at n = 8192, b = 128: reserving 96
// rather than 64 CUs costs the far update little and shortens the panel chain
// (its cross-workgroup exchanges meet less memory traffic).
struct SideStream {
  int dev = -1;
  hipStream_t s = nullptr;
  hipStream_t main = nullptr;   // panel chain of LU_PRRP, on the reserved CUs
  hipStream_t main_any = nullptr;   // panel chain of CALU_PRRP: a tournament level
                                    // may hold more workgroups than the reserve
  hipStream_t s2 = nullptr;     // GEPP / L21 / U12 of finished panels
  hipEvent_t ev[64] = {};
  int next = 0;
  int main_cus = 0;             // CUs `main` is confined to (0: all)
};
SideStream g_side;

bool lookahead_enabled() {
  static int on = -1;
  if (on < 0) {
    const char* e = getenv("PRRP_LOOKAHEAD");
    on = (e && atoi(e) == 0) ? 0 : 1;
  }
  return on == 1;
}

hipError_t side_stream(hipStream_t* out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (g_side.s && g_side.dev == dev) { *out = g_side.s; return hipSuccess; }
  const char* env = getenv("PRRP_RESERVE_CUS");
  int cus = 0;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  int reserve = env ? atoi(env) : 96;
  if (reserve < 0) reserve = 0;
  if (reserve > cus / 2) reserve = cus / 2;
  std::vector<uint32_t> mask((cus + 31) / 32, 0u);
  for (int c = 0; c < cus - reserve; ++c) mask[c / 32] |= 1u << (c % 32);
  hipStream_t s = nullptr;
  if (reserve == 0 ||
      hipExtStreamCreateWithCUMask(&s, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  for (auto& ev : g_side.ev) {
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) return e;
  }
  // The panel chain keeps to the reserved CUs (PRRP_MAIN_MASK=0: anywhere),
  // so its persistent strong-RRQR workgroups never share a SIMD with the far
  // update.  The mask interleaves over the XCDs, so every XCD keeps
  // reserve / 8 CUs for it.
  const char* em = getenv("PRRP_MAIN_MASK");
  const bool main_mask = reserve > 0 && !(em && atoi(em) == 0);
  std::vector<uint32_t> mmask((cus + 31) / 32, 0u);
  for (int c = cus - reserve; c < cus; ++c) mmask[c / 32] |= 1u << (c % 32);
  g_side.main_cus = 0;
  if (main_mask &&
      hipExtStreamCreateWithCUMask(&g_side.main, (uint32_t)mmask.size(), mmask.data()) == hipSuccess) {
    g_side.main_cus = reserve;
  } else {
    e = hipStreamCreateWithFlags(&g_side.main, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  e = hipStreamCreateWithFlags(&g_side.main_any, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  e = hipStreamCreateWithFlags(&g_side.s2, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  g_side.s = s;
  g_side.dev = dev;
  *out = s;
  return hipSuccess;
}

hipEvent_t side_event() {
  hipEvent_t e = g_side.ev[g_side.next];
  g_side.next = (g_side.next + 1) & 63;
  return e;
}

// ------------------------------------------------------------ phase timer
struct PhaseTimer {
  bool on = false;
  struct Rec { int phase; hipEvent_t a, b; };
  std::vector<Rec> recs;
  std::vector<hipEvent_t> pool;
  double ms[PRRP_PHASES] = {0};
  int64_t count[PRRP_PHASES] = {0};
  hipEvent_t get() {
    if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  void drain() {
    for (auto& r : recs) {
      float t = 0.f;
      if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.phase] += t;
        count[r.phase] += 1;
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    recs.clear();
  }
};
PhaseTimer g_timer;

// Scope that brackets one launch with events when the timer is on.
struct PhaseScope {
  int phase; hipStream_t st; hipEvent_t a = nullptr, b = nullptr;
  PhaseScope(int p, hipStream_t s) : phase(p), st(s) {
    if (g_timer.on) { a = g_timer.get(); if (a) (void)hipEventRecord(a, st); }
  }
  ~PhaseScope() {
    if (g_timer.on && a) {
      b = g_timer.get();
      if (b) { (void)hipEventRecord(b, st); g_timer.recs.push_back({phase, a, b}); }
    }
  }
};
#define PRRP_TRY(x)                                   \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return herr(e_);            \
  } while (0)

struct Ctx {
  double* A;
  int64_t n, lda;
  int b;
  double tau;
  int64_t* perm;
  prrp_stats* stats;
  char* ws;
  Layout L;
  hipStream_t st;
  int schur;
  // slot bookkeeping across srrqr launches
  int launch_no = 0;
  uint64_t* prev_base = nullptr;
  size_t prev_group_stride = 0;
  int prev_ngroups = 0, prev_G = 0, prev_bw = 0;
  int32_t* prev_rounds = nullptr;
  int cap = 256;
  int rpw_target = 64;               // rows per panel workgroup (64 or 128)
  hipStream_t side = nullptr;        // look-ahead stream (null: no look-ahead)
  hipStream_t side2 = nullptr;       // GEPP / L21 / U12 stream (null: no look-ahead)
  hipEvent_t far_event = nullptr;    // pending far Schur update on `side`
  int pidx = 0;                      // panel index (parity of sel / Y)
  // The previous panel's GEPP path past its last reads of sel, Y, the moves
  // and its panel buffer, and past the far update (which it waits for).
  hipEvent_t join_event = nullptr;
  const double* panel_src = nullptr; // this panel's columns (null: in A)

  uint64_t* slot_set(int parity) {
    return reinterpret_cast<uint64_t*>(ws + L.off_slots) + (size_t)parity * L.slots_set_words;
  }
  int32_t* rounds(int parity) {
    return reinterpret_cast<int32_t*>(ws + L.off_rounds) + (size_t)parity * L.max_groups;
  }
  uint32_t* abort_flag() { return reinterpret_cast<uint32_t*>(ws + L.off_abort); }
  // sel and Y alternate between panels: the next panel's strong RRQR writes
  // one pair while the previous panel's GEPP, L21 and far update read the other
  int32_t* sel() {
    return reinterpret_cast<int32_t*>(ws + L.off_sel) + (size_t)(pidx & 1) * L.sel_stride;
  }
  int32_t* lsel() { return reinterpret_cast<int32_t*>(ws + L.off_lsel); }
  int32_t* lists() { return reinterpret_cast<int32_t*>(ws + L.off_lists); }
  double* Y() { return reinterpret_cast<double*>(ws + L.off_y + (size_t)(pidx & 1) * L.y_stride); }
  double* PL() { return reinterpret_cast<double*>(ws + L.off_pl); }
  int32_t* p11() { return reinterpret_cast<int32_t*>(ws + L.off_p11); }
  // the move lists alternate too: the far and left moves of a panel run on
  // the side streams while the next panel's plan writes the other list
  double* panel_buf(int parity) {
    return reinterpret_cast<double*>(ws + L.off_panel + (size_t)parity * L.panel_stride);
  }
  int32_t* srcmap() { return reinterpret_cast<int32_t*>(ws + L.off_srcmap); }
  double* winv() { return reinterpret_cast<double*>(ws + L.off_winv); }
  // this panel's Y rows sit at their positions after the moves (the moves
  // must not carry them again)
  bool y_final = false;

  // CALU_PRRP after the tournament (Section 3.1): the winners become the
  // panel's pivots and L_2j = A21 A11^-1, which equals (R11^-1 R12)^T of the
  // QR without pivoting of the panel transpose with the winners first.  No
  // step here waits on another workgroup: the moves and the source-row map,
  // the inverse of the b x b block (one workgroup), and one gathered GEMM
  // that writes Y at the rows' positions after the moves.
  hipError_t calu_root(int64_t k0, int bw, const int32_t* winners) {
    const int64_t m = n - k0;
    GeppArgs ga{A, lda, k0, bw, (int)m, sel(), PL(), mv(), mv() + 2 * kMaxB, mv() + 4 * kMaxB,
                stats, p11(), panel_src, b};
    PhaseScope ps(0, st);
    hipError_t e = launch_root(ga, winners, sel(), srcmap(), winv(), st);
    if (e != hipSuccess) return e;
    if (m > bw) {
      GemmArgs y{(int)(m - bw), bw, bw, panel_src ? panel_src : A + k0 * lda + k0,
                 panel_src ? (int64_t)b : lda, winv(), bw, Y() + (size_t)bw * b, b, 1.0, 0.0,
                 &stats->max_block_L, nullptr, PRRP_FP64};
      y.a_rows = srcmap();
      y.gather_rows = (int)m;
      e = launch_gemm(y, st);
      if (e != hipSuccess) return e;
    }
    y_final = true;
    return hipSuccess;
  }
  int32_t* mv() {
    return reinterpret_cast<int32_t*>(ws + L.off_moves +
                                      (size_t)(pidx & 1) * align_up((size_t)(4 * kMaxB + 4) * 4, 256));
  }

  // One srrqr launch; fills in the slot-set bookkeeping.
  hipError_t srrqr(SrrqrArgs& a) {
    const int parity = launch_no & 1;
    a.slots = slot_set(parity);
    a.group_stride = (size_t)kRoundsMax * a.G * kPostW;
    a.rounds_out = rounds(parity);
    a.clear_base = prev_base;
    a.clear_group_stride = prev_group_stride;
    a.clear_ngroups = prev_ngroups;
    a.clear_G = prev_G;
    a.clear_bw = prev_bw;
    a.clear_rounds = prev_rounds;
    a.stats = stats;
    a.abort_flag = abort_flag();
    a.tau_bits = tau_bits(tau);
    // Tiles interleaved over the XCDs when the whole launch fits the CUs it
    // can count on: the device, or while far updates run on the side stream
    // the CUs reserved from them.  A launch that only partly fits, with its
    // tiles interleaved, holds some workgroups of every tile resident and
    // no tile can finish until the far update does (measured: 12 ms at an
    // early panel of CALU_PRRP at n = 16384); in tile order the resident
    // tiles finish and free their CUs for the rest.
    if (a.ngroups > 1 && a.G > 1 && interleave_tiles()) {
      const int64_t cus = tile_cus(a.G, a.bw, a.rpw, 0, (int64_t)a.ngroups * a.G);
      const int64_t room = (side != nullptr && g_side.main_cus > 0) ? g_side.main_cus : device_cus();
      a.interleave = (cus > 0 && cus <= room) ? 1 : 0;
    }
    hipError_t e;
    {
      PhaseScope ps(0, st);
      e = launch_srrqr(a, st);
    }
    prev_base = a.slots;
    prev_group_stride = a.group_stride;
    prev_ngroups = a.ngroups;
    prev_G = a.G;
    prev_bw = a.bw;
    prev_rounds = a.rounds_out;
    ++launch_no;
    return e;
  }

  // Steps after the pivot rows of the panel at k0 are known (sel(), Y()).
  //
  // The trailing update is the block form of Algorithm "LU_PRRP
  // factorization", A22 -= L_2j A12 with L_2j = M^T (Y) and A12 before the
  // diagonal GEPP.
  //
  // With look-ahead the strong RRQR has already formed the moves of Pi_j and
  // written M^T in the order after them.  Critical path (stream st): the
  // update of the next panel's columns, gathered from their rows before the
  // moves and written to a panel buffer, which is all the next panel reads.
  // `side`: the far columns' moves and update.  `side2`: the moves of the
  // columns left of the panel and of perm, GEPP of the diagonal block, Pi11 on
  // the left columns and perm, the stored L21 = M^T Pi11 L11, the moves of the
  // top rows in the next panel's columns, and U12 = L11^-1 Pi11^T A12.
  // Without look-ahead all of it runs in order on st, moves first.
  hipError_t finish_panel(int64_t k0, int bw) {
    const int64_t m = n - k0;
    int32_t* mv_dst = mv();
    int32_t* mv_src = mv() + 2 * kMaxB;
    int32_t* n_moves = mv() + 4 * kMaxB;
    double* Yp = Y();
    const bool la = side2 != nullptr;
    GeppArgs ga{A, lda, k0, bw, (int)m, sel(), PL(), mv_dst, mv_src, n_moves, stats, p11(),
                panel_src, b};
    hipError_t e;
    const int64_t nr = n - k0 - bw;
    double* a12 = A + k0 * lda + k0 + bw;
    double* a22 = A + (k0 + bw) * lda + k0 + bw;
    const double* yrest = Yp + (size_t)bw * b;
    hipStream_t gs = la ? side2 : st;
    hipEvent_t ev_near = nullptr, ev_far = nullptr;
    int64_t n_near = nr;
    double* next_panel = nullptr;
    if (!la) {
      {
        PhaseScope ps(2, st);
        e = launch_plan(ga, st);
      }
      if (e != hipSuccess) return e;
      MoveArgs ma{A, lda, n, k0, bw, mv_dst, mv_src, n_moves, perm,
                  (m > bw && !y_final) ? Yp : nullptr, b, 0, n, k0, bw, 0};
      {
        PhaseScope ps(2, st);
        e = launch_moves(ma, st);
      }
      if (e != hipSuccess) return e;
      if (m > bw) {
        GemmArgs sc{(int)(m - bw), (int)nr, bw, yrest, b, a12, lda, a22, lda, -1.0, 1.0,
                    &stats->max_abs_W, nullptr, schur};
        {
          PhaseScope ps(5, st);
          e = launch_gemm(sc, st);
        }
        if (e != hipSuccess) return e;
      }
    } else {
      // One event on the panel chain per panel, after the near update (or
      // after the strong RRQR when there is none): both side streams start
      // from it, which keeps a second marker out of the critical path.  A far
      // update long enough to outlast the next strong RRQR starts right after
      // this one instead (an extra marker): at FP64, (m - b) x far columns
      // above 36 M elements (72 M with FP32 / BF16 operands), measured at
      // about 20 and 40 TFLOP/s against about 4.5 us per strong-RRQR step.
      const int64_t nfar = (m > bw) ? nr - std::min<int64_t>(b, nr) : 0;
      const double far_area = (double)(m - bw) * (double)nfar;
      static const double early_area = [] {
        const char* v = getenv("PRRP_FAR_EARLY_AREA");   // FP64 threshold, elements
        return v ? atof(v) : 3.6e7;
      }();
      const bool far_early =
          nfar > 0 && far_area > ((schur == PRRP_FP64) ? early_area : 2.0 * early_area);
      hipEvent_t ev_sel = nullptr;
      if (far_early) {
        ev_sel = side_event();
        e = hipEventRecord(ev_sel, st);
        if (e != hipSuccess) return e;
      }
      if (m > bw) {
        n_near = std::min<int64_t>(b, nr);
        // One wait: the previous far update wrote these columns, the
        // previous panel's GEPP read the buffer written here, and the strong
        // RRQR of the next panel reuses the buffers (sel, Y, moves) of the
        // panel before this one, whose readers all precede that event.
        if (join_event != nullptr) {
          e = hipStreamWaitEvent(st, join_event, 0);
          if (e != hipSuccess) return e;
          join_event = nullptr;
        }
        next_panel = panel_buf((pidx + 1) & 1);
        const double* near = A + k0 * lda + k0 + bw;     // panel row 0 of these columns
        GemmArgs sc{(int)(m - bw), (int)n_near, bw, yrest, b, near, lda, next_panel, b, -1.0,
                    1.0, &stats->max_abs_W, nullptr, schur, sel(), near, lda, srcmap(), (int)m};
        {
          PhaseScope ps(5, st);
          e = launch_gemm(sc, st);
        }
        if (e != hipSuccess) return e;
      }
      ev_near = side_event();
      e = hipEventRecord(ev_near, st);
      if (e != hipSuccess) return e;
      if (m > bw) {
        if (nr > n_near) {
          e = hipStreamWaitEvent(side, far_early ? ev_sel : ev_near, 0);
          if (e != hipSuccess) return e;
          MoveArgs mf{A, lda, n, k0, bw, mv_dst, mv_src, n_moves, nullptr, nullptr, b,
                      k0 + bw + n_near, n, n, 0, 0};
          {
            PhaseScope ps(2, side);
            e = launch_moves(mf, side);
          }
          if (e != hipSuccess) return e;
          GemmArgs sc_far{(int)(m - bw), (int)(nr - n_near), bw, yrest, b, a12 + n_near, lda,
                          a22 + n_near, lda, -1.0, 1.0, &stats->max_abs_W, nullptr, schur};
          {
            PhaseScope ps(5, side);
            e = launch_gemm(sc_far, side);
          }
          if (e != hipSuccess) return e;
          ev_far = side_event();
          e = hipEventRecord(ev_far, side);
          if (e != hipSuccess) return e;
          far_event = ev_far;
        }
      }
      // ---- GEPP path
      e = hipStreamWaitEvent(gs, ev_near, 0);
      if (e != hipSuccess) return e;
      if (k0 > 0 || perm != nullptr) {
        MoveArgs ml{A, lda, n, k0, bw, mv_dst, mv_src, n_moves, perm, nullptr, b, 0, k0, n, 0, 0};
        {
          PhaseScope ps(2, gs);
          e = launch_moves(ml, gs);
        }
        if (e != hipSuccess) return e;
      }
    }
    {
      PhaseScope ps(1, gs);
      e = launch_gepp(ga, gs);
    }
    if (e != hipSuccess) return e;
    PermTopArgs pt{A, lda, k0, bw, perm, p11()};
    {
      PhaseScope ps(1, gs);
      e = launch_perm_top(pt, gs);
    }
    if (e != hipSuccess) return e;
    if (m > bw) {
      // L21 = M^T (Pi11 L11)
      GemmArgs l21{(int)(m - bw), bw, bw, yrest, b, PL(), bw, A + (k0 + bw) * lda + k0, lda, 1.0,
                   0.0, nullptr, nullptr, PRRP_FP64};
      {
        PhaseScope ps(3, gs);
        e = launch_gemm(l21, gs);
      }
      if (e != hipSuccess) return e;
      if (la) {
        // top rows of the next panel's columns (the near update has read them)
        MoveArgs mt{A, lda, n, k0, bw, mv_dst, mv_src, n_moves, nullptr, nullptr, b,
                    k0 + bw, k0 + bw + n_near, n, 0, 1};
        {
          PhaseScope ps(2, gs);
          e = launch_moves(mt, gs);
        }
        if (e != hipSuccess) return e;
        if (ev_far != nullptr) {
          e = hipStreamWaitEvent(gs, ev_far, 0);
          if (e != hipSuccess) return e;
        }
        join_event = side_event();
        e = hipEventRecord(join_event, gs);
        if (e != hipSuccess) return e;
      }
      {
        PhaseScope ps(4, gs);
        e = launch_trsm_u12(A, lda, k0, bw, nr, &stats->max_abs_U, &stats->max_abs_W, p11(), gs);
      }
      if (e != hipSuccess) return e;
    }
    panel_src = next_panel;
    y_final = false;
    ++pidx;
    return hipSuccess;
  }
};

SrrqrArgs base_args(Ctx& c, int64_t k0, int bw) {
  SrrqrArgs a;
  std::memset(&a, 0, sizeof a);
  a.A = c.A;
  a.lda = c.lda;
  a.k0 = k0;
  a.bw = bw;
  a.ldy = c.b;
  a.panel = c.panel_src;
  a.ldp = c.b;
  return a;
}

int validate_common(double* A, int64_t n, int64_t lda, int b, double tau, int64_t* perm,
                    prrp_stats* stats, void* ws) {
  if (!A) return -1;
  if (n < 1 || n > kMaxN) return -2;
  if (lda < n) return -3;
  if (b < 1 || b > kMaxB || b > n) return -4;
  if (!(tau > 1.0) || !std::isfinite(tau)) return -5;
  if (!perm) return -6;
  if (!stats) return -7;
  if (!ws) return -8;
  return 0;
}

// The most compute units any tile of any strong-RRQR launch of this
// factorization needs at once (-1: occupancy query failed).
int64_t factor_tile_cus(int method, int64_t n, int b, int tree, int64_t tile_rows, int cap,
                        int rpw_target, int bpc_given = 0) {
  int64_t need = 0;
  auto one = [&](int64_t rows, int bw) {
    const int G = groups_for_rows(rows, cap, rpw_target, bw);
    const int rpw = (int)((rows + G - 1) / G);
    const int64_t c = tile_cus(G, bw, rpw, bpc_given);
    need = (c < 0 || need < 0) ? -1 : std::max(need, c);
  };
  for (int64_t k0 = 0; k0 < n && need >= 0; k0 += b) {
    const int bw = (int)std::min<int64_t>(b, n - k0);
    const int64_t m = n - k0;
    if (method == 0) { one(m, bw); continue; }
    const Tiles t = tile_bounds(m, tile_rows, bw);
    if (t.start.size() == 1) { one(m, bw); continue; }   // one tile: LU_PRRP's panel
    int maxlen = 0;
    for (int l : t.len) maxlen = std::max(maxlen, l);
    if (tree == PRRP_TREE_BINARY) {
      one(maxlen, bw);
      one(2 * bw, bw);
    } else {
      one(t.len[0], bw);
      for (size_t i = 1; i < t.len.size(); ++i) one(bw + t.len[i], bw);
    }
  }
  return need;
}

int run_factor(int method, double* A, int64_t n, int64_t lda, int b, double tau, int tree,
               int64_t tile_rows, int64_t* perm, prrp_stats* stats, void* workspace,
               size_t ws_bytes, void* stream, int schur, bool lookahead = true,
               int rpw_target = 64) {
  Ctx c;
  c.rpw_target = rpw_target;
  c.A = A; c.n = n; c.lda = lda; c.b = b; c.tau = tau; c.perm = perm; c.stats = stats;
  c.ws = static_cast<char*>(workspace);
  c.st = static_cast<hipStream_t>(stream);
  c.schur = schur;
  c.cap = std::min(256, device_cus());
  c.L = make_layout(n, b, method, tile_rows);
  PRRP_TRY(srrqr_prepare());
  // every workgroup of a strong-RRQR tile waits on the others: a tile that
  // the device cannot hold at once is an argument error, found here
  const int64_t need_cus = factor_tile_cus(method, n, b, tree, tile_rows, c.cap, c.rpw_target);
  if (need_cus < 0) return herr(hipErrorInvalidValue);
  if (need_cus > device_cus()) return method == 0 ? -2 : -7;
  hipStream_t caller = c.st;
  // The look-ahead streams and their event ring are shared by the process:
  // one host thread at a time enqueues a factorization on them.
  static std::mutex lookahead_mu;
  std::unique_lock<std::mutex> lock(lookahead_mu, std::defer_lock);
  if (lookahead && lookahead_enabled() && n > 2 * b) {
    lock.lock();
    // The panel chain runs on an internal non-blocking stream and the far
    // Schur updates on the side stream; both start after earlier work on the
    // caller's stream, which in turn waits for both at the end.
    PRRP_TRY(side_stream(&c.side));
    hipEvent_t e0 = side_event();
    PRRP_TRY(hipEventRecord(e0, caller));
    PRRP_TRY(hipStreamWaitEvent(c.side, e0, 0));
    // the panel chain keeps to the reserved CUs when every strong-RRQR tile
    // of the factorization fits them (a CALU_PRRP tournament level spans
    // several tiles, which need not be resident together)
    const bool fits = g_side.main_cus == 0 || need_cus <= g_side.main_cus;
    hipStream_t chain = (method == 0 && fits) ? g_side.main : g_side.main_any;
    PRRP_TRY(hipStreamWaitEvent(chain, e0, 0));
    PRRP_TRY(hipStreamWaitEvent(g_side.s2, e0, 0));
    c.st = chain;
    c.side2 = g_side.s2;
  }
  int height = 0;
  if (method == 1) {
    // tallest tournament: the first panel has the most tiles
    const Tiles t0 = tile_bounds(n, tile_rows, std::min<int64_t>(b, n));
    const int nt = (int)t0.start.size();
    if (tree == PRRP_TREE_BINARY) { while ((1 << height) < nt) ++height; }
    else height = nt - 1;
  }
  {
    PhaseScope ps(6, c.st);
    PRRP_TRY(launch_init_factor(A, n, lda, perm, stats, c.abort_flag(), height,
                                (int)((n + b - 1) / b), c.st));
    PRRP_TRY(launch_fill_u64(c.slot_set(0), 2 * c.L.slots_set_words, kKeySent, c.st));
  }

  for (int64_t k0 = 0; k0 < n; k0 += b) {
    const int bw = (int)std::min<int64_t>(b, n - k0);
    const int64_t m = n - k0;
    Tiles t;
    if (method == 1) t = tile_bounds(m, tile_rows, bw);
    if (method == 0 || t.start.size() == 1) {
      SrrqrArgs a = base_args(c, k0, bw);
      a.ngroups = 1;
      a.G = groups_for_rows(m, c.cap, c.rpw_target, bw);
      a.rpw = (int)((m + a.G - 1) / a.G);
      a.tile_start[0] = 0;
      a.tile_len[0] = (int)m;
      a.report_rank = 1;
      a.record_block_L = 1;
      a.sel_out = c.sel();
      a.Y = (m > bw) ? c.Y() : nullptr;
      if (c.side2 != nullptr) { a.plan_mv = c.mv(); a.srcmap = c.srcmap(); }
      PRRP_TRY(c.srrqr(a));
    } else {
      // ---------------------------------------------- tournament (Sec. 3.1)
      const int ntiles = (int)t.start.size();
      if (ntiles > kMaxGroups) return -9;
      int maxlen = 0;
      for (int l : t.len) maxlen = std::max(maxlen, l);
      int32_t* cur = c.lsel();        // candidate sets of the current level
      int32_t* nxt = c.lsel() + (size_t)c.L.max_groups * kMaxB;
      int32_t* lists = c.lists();
      if (tree == PRRP_TREE_BINARY) {
        SrrqrArgs a = base_args(c, k0, bw);
        a.ngroups = ntiles;
        a.G = groups_for_rows(maxlen, c.cap, c.rpw_target, bw);
        a.rpw = (maxlen + a.G - 1) / a.G;
        for (int i = 0; i < ntiles; ++i) { a.tile_start[i] = t.start[i]; a.tile_len[i] = t.len[i]; }
          a.sel_out = cur;
        PRRP_TRY(c.srrqr(a));
        int level = ntiles;
        while (level > 1) {
          const int pairs = level / 2;
          // lists of stacked pairs; an odd last node is promoted into cur[pairs]
          PRRP_TRY(launch_build_lists(cur, level, bw, lists, nxt, pairs, -1, 0, c.st));
          SrrqrArgs nd = base_args(c, k0, bw);
          nd.ngroups = pairs;
          nd.G = groups_for_rows(2 * bw, c.cap, c.rpw_target, bw);
          nd.rpw = (2 * bw + nd.G - 1) / nd.G;
          for (int i = 0; i < pairs; ++i) { nd.tile_start[i] = i * 2 * bw; nd.tile_len[i] = 2 * bw; }
          nd.row_list = lists;
          nd.sel_out = nxt;
          PRRP_TRY(c.srrqr(nd));
          level = pairs + (level & 1);
          std::swap(cur, nxt);
        }
      } else {
        // flat tree: running candidates stacked over each next whole tile
        SrrqrArgs a = base_args(c, k0, bw);
        a.ngroups = 1;
        a.G = groups_for_rows(t.len[0], c.cap, c.rpw_target, bw);
        a.rpw = (t.len[0] + a.G - 1) / a.G;
        a.tile_start[0] = t.start[0];
        a.tile_len[0] = t.len[0];
          a.sel_out = cur;
        PRRP_TRY(c.srrqr(a));
        for (int i = 1; i < ntiles; ++i) {
          PRRP_TRY(launch_build_lists(cur, 1, bw, lists, nullptr, 1, t.start[i], t.len[i], c.st));
          SrrqrArgs nd = base_args(c, k0, bw);
          const int len = bw + t.len[i];
          nd.ngroups = 1;
          nd.G = groups_for_rows(len, c.cap, c.rpw_target, bw);
          nd.rpw = (len + nd.G - 1) / nd.G;
          nd.tile_start[0] = 0;
          nd.tile_len[0] = len;
          nd.row_list = lists;
          nd.sel_out = nxt;
          PRRP_TRY(c.srrqr(nd));
          std::swap(cur, nxt);
        }
      }
      // the winners become the panel's pivots
      PRRP_TRY(c.calu_root(k0, bw, cur));
    }
    PRRP_TRY(c.finish_panel(k0, bw));
  }
  if (c.far_event != nullptr) PRRP_TRY(hipStreamWaitEvent(c.st, c.far_event, 0));
  if (c.side2 != nullptr) {
    hipEvent_t e2 = side_event();
    PRRP_TRY(hipEventRecord(e2, c.side2));
    PRRP_TRY(hipStreamWaitEvent(c.st, e2, 0));
  }
  if (c.st != caller) {
    hipEvent_t e1 = side_event();
    PRRP_TRY(hipEventRecord(e1, c.st));
    PRRP_TRY(hipStreamWaitEvent(caller, e1, 0));
  }
  return 0;
}

// ------------------------------------- block parallel / block pairwise LU_PRRP
// Section 5 and Appendix E: the CALU_PRRP workspace plus the lists of each
// level's left-out rows, the level's GEMM arguments, an identity selection
// (the diagonal GEPP reads the top block after whole-row moves), and the node
// records kept by original row until the end.
struct BlockLayout {
  Layout L;
  int panels = 0, max_nodes = 0, elim_stride = 0;
  size_t off_elim = 0, off_list = 0, off_iota = 0, off_nsel = 0, off_nelim = 0, off_counts = 0,
         off_inv = 0, total = 0;
};

int block_max_nodes(int64_t n, int b, int tree, int64_t tile_rows) {
  const int64_t nt = (int64_t)tile_bounds(n, tile_rows, (int)std::min<int64_t>(b, n)).start.size();
  if (nt <= 1) return 1;
  return (int)(tree == PRRP_TREE_BINARY ? 2 * nt - 1 : nt);
}

BlockLayout make_block_layout(int64_t n, int b, int tree, int64_t tile_rows) {
  BlockLayout B;
  B.L = make_layout(n, b, 1, tile_rows);
  B.panels = (int)((n + b - 1) / b);
  B.max_nodes = block_max_nodes(n, b, tree, tile_rows);
  // the longest node: a tile with the remainder it absorbed, or a flat-tree
  // node (b candidates over a tile)
  B.elim_stride = (int)std::min<int64_t>(n, tile_rows + 2 * (int64_t)b);
  size_t off = align_up(B.L.total, 256);
  B.off_elim = off;   off += align_up((size_t)kMaxGroups * B.elim_stride * 4, 256);
  B.off_list = off;   off += align_up((size_t)kMaxGroups * sizeof(GemmArgs), 256);
  B.off_iota = off;   off += align_up((size_t)kMaxB * 4, 256);
  B.off_nsel = off;   off += align_up((size_t)B.panels * B.max_nodes * kMaxB * 4, 256);
  B.off_nelim = off;  off += align_up((size_t)B.panels * n * 4, 256);
  B.off_counts = off; off += align_up((size_t)B.panels * 4, 256);
  B.off_inv = off;    off += align_up((size_t)n * 4, 256);
  B.total = off;
  return B;
}

int64_t block_nodes_len(int64_t n, int b, int tree, int64_t tile_rows) {
  const int64_t P = (n + b - 1) / b;
  return 2 + P + P * block_max_nodes(n, b, tree, tile_rows) * (int64_t)b + P * n;
}

int run_block_factor(double* A, int64_t n, int64_t lda, int b, double tau, int tree,
                     int64_t tile_rows, int64_t* perm, int32_t* nodes, prrp_stats* stats,
                     void* workspace, void* stream) {
  Ctx c;
  c.A = A; c.n = n; c.lda = lda; c.b = b; c.tau = tau; c.perm = perm; c.stats = stats;
  c.ws = static_cast<char*>(workspace);
  c.st = static_cast<hipStream_t>(stream);
  c.schur = PRRP_FP64;
  c.cap = std::min(256, device_cus());
  const BlockLayout BL = make_block_layout(n, b, tree, tile_rows);
  c.L = BL.L;
  PRRP_TRY(srrqr_prepare());
  const int64_t need_cus = factor_tile_cus(1, n, b, tree, tile_rows, c.cap, c.rpw_target);
  if (need_cus < 0) return herr(hipErrorInvalidValue);
  if (need_cus > device_cus()) return -7;
  char* ws = c.ws;
  int32_t* elim = reinterpret_cast<int32_t*>(ws + BL.off_elim);
  GemmArgs* list = reinterpret_cast<GemmArgs*>(ws + BL.off_list);
  int32_t* iota = reinterpret_cast<int32_t*>(ws + BL.off_iota);
  int32_t* nsel = reinterpret_cast<int32_t*>(ws + BL.off_nsel);
  int32_t* nelim = reinterpret_cast<int32_t*>(ws + BL.off_nelim);
  int32_t* counts = reinterpret_cast<int32_t*>(ws + BL.off_counts);
  int32_t* inv = reinterpret_cast<int32_t*>(ws + BL.off_inv);
  const int MN = BL.max_nodes;
  int height = 0;
  {
    const Tiles t0 = tile_bounds(n, tile_rows, (int)std::min<int64_t>(b, n));
    const int nt = (int)t0.start.size();
    if (tree == PRRP_TREE_BINARY) { while ((1 << height) < nt) ++height; }
    else height = nt - 1;
  }
  PRRP_TRY(launch_init_factor(A, n, lda, perm, stats, c.abort_flag(), height, BL.panels, c.st));
  PRRP_TRY(launch_fill_u64(c.slot_set(0), 2 * c.L.slots_set_words, kKeySent, c.st));
  PRRP_TRY(launch_fill_i32(iota, kMaxB, 0, 1, c.st));
  PRRP_TRY(launch_fill_i32(nsel, (int64_t)BL.panels * MN * kMaxB, -1, 0, c.st));
  PRRP_TRY(launch_fill_i32(nelim, (int64_t)BL.panels * n, -1, 0, c.st));
  PRRP_TRY(launch_fill_i32(counts, BL.panels, 0, 0, c.st));

  for (int64_t k0 = 0, j = 0; k0 < n; k0 += b, ++j) {
    const int bw = (int)std::min<int64_t>(b, n - k0);
    const int64_t m = n - k0;
    int node0 = 0;
    // a level's strong RRQR (d_r of every left-out row into its panel
    // columns), then its nodes' records and in-place updates
    auto level = [&](SrrqrArgs& a) -> int {
      a.Y = A + k0 * lda + k0;
      a.ldy = lda;
      a.report_rank = 1;
      a.record_block_L = 1;
      PRRP_TRY(c.srrqr(a));
      BlockNodeArgs nb{A, lda, k0, n, (int)m, node0, elim, BL.elim_stride, perm,
                       nsel + (size_t)j * MN * kMaxB, nelim + (size_t)j * n, counts + j, list,
                       &stats->max_abs_W};
      PRRP_TRY(launch_block_nodes(a, nb, c.st));
      int max_m = 0;
      for (int g = 0; g < a.ngroups; ++g) max_m = std::max(max_m, a.tile_len[g] - bw);
      const int64_t nr = n - k0 - bw;
      if (max_m > 0 && nr > 0) {
        PhaseScope ps(5, c.st);
        PRRP_TRY(launch_gemm_batched(list, a.ngroups, max_m, (int)nr, PRRP_FP64, c.st));
      }
      node0 += a.ngroups;
      return 0;
    };
    Tiles t;
    if (m > bw) t = tile_bounds(m, tile_rows, bw);
    int32_t* cur = c.lsel();
    int32_t* nxt = c.lsel() + (size_t)c.L.max_groups * kMaxB;
    int32_t* lists = c.lists();
    if (m <= bw || t.start.size() == 1) {
      SrrqrArgs a = base_args(c, k0, bw);
      a.ngroups = 1;
      a.G = groups_for_rows(m, c.cap, c.rpw_target, bw);
      a.rpw = (int)((m + a.G - 1) / a.G);
      a.tile_start[0] = 0;
      a.tile_len[0] = (int)m;
      a.sel_out = cur;
      if (int rc = level(a)) return rc;
    } else {
      const int ntiles = (int)t.start.size();
      if (ntiles > kMaxGroups) return -7;
      int maxlen = 0;
      for (int l : t.len) maxlen = std::max(maxlen, l);
      if (tree == PRRP_TREE_BINARY) {
        SrrqrArgs a = base_args(c, k0, bw);
        a.ngroups = ntiles;
        a.G = groups_for_rows(maxlen, c.cap, c.rpw_target, bw);
        a.rpw = (maxlen + a.G - 1) / a.G;
        for (int i = 0; i < ntiles; ++i) { a.tile_start[i] = t.start[i]; a.tile_len[i] = t.len[i]; }
        a.sel_out = cur;
        if (int rc = level(a)) return rc;
        int lv = ntiles;
        while (lv > 1) {
          const int pairs = lv / 2;
          PRRP_TRY(launch_build_lists(cur, lv, bw, lists, nxt, pairs, -1, 0, c.st));
          SrrqrArgs nd = base_args(c, k0, bw);
          nd.ngroups = pairs;
          nd.G = groups_for_rows(2 * bw, c.cap, c.rpw_target, bw);
          nd.rpw = (2 * bw + nd.G - 1) / nd.G;
          for (int i = 0; i < pairs; ++i) { nd.tile_start[i] = i * 2 * bw; nd.tile_len[i] = 2 * bw; }
          nd.row_list = lists;
          nd.sel_out = nxt;
          if (int rc = level(nd)) return rc;
          lv = pairs + (lv & 1);
          std::swap(cur, nxt);
        }
      } else {
        SrrqrArgs a = base_args(c, k0, bw);
        a.ngroups = 1;
        a.G = groups_for_rows(t.len[0], c.cap, c.rpw_target, bw);
        a.rpw = (t.len[0] + a.G - 1) / a.G;
        a.tile_start[0] = t.start[0];
        a.tile_len[0] = t.len[0];
        a.sel_out = cur;
        if (int rc = level(a)) return rc;
        for (int i = 1; i < ntiles; ++i) {
          PRRP_TRY(launch_build_lists(cur, 1, bw, lists, nullptr, 1, t.start[i], t.len[i], c.st));
          SrrqrArgs nd = base_args(c, k0, bw);
          const int len = bw + t.len[i];
          nd.ngroups = 1;
          nd.G = groups_for_rows(len, c.cap, c.rpw_target, bw);
          nd.rpw = (len + nd.G - 1) / nd.G;
          nd.tile_start[0] = 0;
          nd.tile_len[0] = len;
          nd.row_list = lists;
          nd.sel_out = nxt;
          if (int rc = level(nd)) return rc;
          std::swap(cur, nxt);
        }
      }
    }
    // the root's rows: Pi_j on entire rows (the panel columns too: they hold
    // the left-out rows' d_r), then GEPP of the top block, Pi11, U12
    GeppArgs gp{A, lda, k0, bw, (int)m, cur, c.PL(), c.mv(), c.mv() + 2 * kMaxB, c.mv() + 4 * kMaxB,
                stats, c.p11(), nullptr, b};
    {
      PhaseScope ps(2, c.st);
      PRRP_TRY(launch_plan(gp, c.st));
      MoveArgs ma{A, lda, n, k0, bw, c.mv(), c.mv() + 2 * kMaxB, c.mv() + 4 * kMaxB, perm, nullptr,
                  b, 0, n, k0, 0, 0};
      PRRP_TRY(launch_moves(ma, c.st));
    }
    GeppArgs gd = gp;
    gd.sel = iota;
    {
      PhaseScope ps(1, c.st);
      PRRP_TRY(launch_gepp(gd, c.st));
      PermTopArgs pt{A, lda, k0, bw, perm, c.p11()};
      PRRP_TRY(launch_perm_top(pt, c.st));
    }
    if (m > bw) {
      PhaseScope ps(4, c.st);
      PRRP_TRY(launch_trsm_u12(A, lda, k0, bw, n - k0 - bw, &stats->max_abs_U, &stats->max_abs_W,
                               c.p11(), c.st));
    }
  }
  BlockRecordArgs ra{perm, n, BL.panels, MN, b, counts, nsel, nelim, inv, nodes};
  PRRP_TRY(launch_block_records(ra, c.st));
  return 0;
}

}  // namespace

extern "C" {

const char* prrp_version(void) { return "prrp-gfx950 0.1"; }

int prrp_profile_enable(int on) {
  g_timer.drain();
  for (int p = 0; p < PRRP_PHASES; ++p) { g_timer.ms[p] = 0.0; g_timer.count[p] = 0; }
  g_timer.on = on != 0;
  return 0;
}

int prrp_profile_read(double* ms, int64_t* launches) {
  g_timer.drain();
  for (int p = 0; p < PRRP_PHASES; ++p) {
    if (ms) ms[p] = g_timer.ms[p];
    if (launches) launches[p] = g_timer.count[p];
  }
  return 0;
}

const char* prrp_status_string(int code) {
  switch (code) {
    case 0: return "success";
    case -1: return "invalid argument 1 (matrix pointer) / info: non-finite value";
    case -2: return "invalid argument 2 (n) / info: bounded wait expired";
    case -3: return "invalid argument 3 (leading dimension) / info: exchange cap reached";
    case -4: return "invalid argument 4 (panel width b)";
    case -5: return "invalid argument 5 (tau must be finite and > 1)";
    default: break;
  }
  if (code <= -1000) return "HIP runtime error while enqueueing";
  if (code < 0) return "invalid argument";
  return "singular: exactly zero residual or pivot at this 1-based column";
}

int prrp_panel_cus(int method, int64_t n, int b, int tree, int64_t tile_rows, int blocks_per_cu,
                   int64_t* cus) {
  if (method != 0 && method != 1) return -1;
  if (n < 1 || n > kMaxN) return -2;
  if (b < 1 || b > kMaxB || b > n) return -3;
  if (method == 1 && tree != PRRP_TREE_BINARY && tree != PRRP_TREE_FLAT) return -4;
  if (method == 1 && tile_rows < b + 1) return -5;
  if (blocks_per_cu < 0) return -6;
  if (!cus) return -7;
  if (blocks_per_cu == 0) {
    const hipError_t e = srrqr_prepare();
    if (e != hipSuccess) return herr(e);
  }
  const int64_t c = factor_tile_cus(method, n, b, tree, method == 1 ? tile_rows : 0,
                                    std::min(256, device_cus()), 64, blocks_per_cu);
  if (c < 0) return herr(hipErrorInvalidValue);
  *cus = c;
  return 0;
}

int prrp_workspace_size(int64_t n, int b, int method, int64_t tile_rows, size_t* bytes) {
  if (n < 1 || n > kMaxN) return -1;
  if (b < 1 || b > kMaxB || b > n) return -2;
  if (method != 0 && method != 1) return -3;
  if (method == 1 && (tile_rows < b + 1)) return -4;
  if (!bytes) return -5;
  *bytes = make_layout(n, b, method, method == 1 ? tile_rows : 0).total;
  return 0;
}

int prrp_factor(double* A, int64_t n, int64_t lda, int b, double tau, int64_t* perm,
                prrp_stats* stats, void* workspace, size_t ws_bytes, void* stream) {
  return prrp_factor_mixed(A, n, lda, b, tau, perm, stats, workspace, ws_bytes, stream, PRRP_FP64);
}

int prrp_factor_mixed(double* A, int64_t n, int64_t lda, int b, double tau, int64_t* perm,
                      prrp_stats* stats, void* workspace, size_t ws_bytes, void* stream,
                      int schur) {
  int v = validate_common(A, n, lda, b, tau, perm, stats, workspace);
  if (v) return v;
  if (ws_bytes < make_layout(n, b, 0, 0).total) return -9;
  if (schur < 0 || schur > 2) return -11;
  return run_factor(0, A, n, lda, b, tau, 0, 0, perm, stats, workspace, ws_bytes, stream, schur);
}

int calu_prrp_factor(double* A, int64_t n, int64_t lda, int b, double tau, int tree,
                     int64_t tile_rows, int64_t* perm, prrp_stats* stats, void* workspace,
                     size_t ws_bytes, void* stream, int schur) {
  if (!A) return -1;
  if (n < 1 || n > kMaxN) return -2;
  if (lda < n) return -3;
  if (b < 1 || b > kMaxB || b > n) return -4;
  if (!(tau > 1.0) || !std::isfinite(tau)) return -5;
  if (tree != PRRP_TREE_BINARY && tree != PRRP_TREE_FLAT) return -6;
  if (tile_rows < b + 1) return -7;
  if (!perm) return -8;
  if (!stats) return -9;
  if (!workspace) return -10;
  if (ws_bytes < make_layout(n, b, 1, tile_rows).total) return -11;
  if (schur < 0 || schur > 2) return -13;
  if ((n + tile_rows - 1) / tile_rows > kMaxGroups) return -7;
  return run_factor(1, A, n, lda, b, tau, tree, tile_rows, perm, stats, workspace, ws_bytes,
                    stream, schur);
}

int prrp_gemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t lda,
              const double* B, int64_t ldb, double beta, double* C, int64_t ldc, int prec,
              void* stream) {
  if (M < 0 || M > INT32_MAX) return -1;
  if (N < 0 || N > INT32_MAX) return -2;
  if (K < 0 || K > INT32_MAX) return -3;
  if (!A && M > 0 && K > 0) return -5;
  if (lda < K) return -6;
  if (!B && K > 0 && N > 0) return -7;
  if (ldb < N) return -8;
  if (!C && M > 0 && N > 0) return -10;
  if (ldc < N) return -11;
  if (prec < 0 || prec > 2) return -12;
  GemmArgs g{(int)M, (int)N, (int)K, A, lda, B, ldb, C, ldc, alpha, beta, nullptr, nullptr, prec};
  return herr(launch_gemm(g, static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------------------ solves
int prrp_solve_workspace_size(int64_t n, int64_t nrhs, size_t* bytes) {
  if (n < 1 || n > kMaxN) return -1;
  if (nrhs < 1) return -2;
  if (!bytes) return -3;
  // tickets | three n x nrhs vectors (two solve buffers, refinement residual) |
  // refinement state | maxima
  *bytes = 256 + 3 * align_up((size_t)n * nrhs * 8, 256) + 256 +
           align_up((size_t)nrhs * 16 + 16, 256);
  return 0;
}

namespace {
struct SolveWs {
  uint32_t* ticket;
  double *t1, *t2, *r, *mx;
  IrState* ir;
  SolveWs(char* ws, int64_t n, int64_t nrhs) {
    const size_t v = align_up((size_t)n * nrhs * 8, 256);
    ticket = reinterpret_cast<uint32_t*>(ws);
    t1 = reinterpret_cast<double*>(ws + 256);
    t2 = reinterpret_cast<double*>(ws + 256 + v);
    r = reinterpret_cast<double*>(ws + 256 + 2 * v);
    ir = reinterpret_cast<IrState*>(ws + 256 + 3 * v);
    mx = reinterpret_cast<double*>(ws + 256 + 3 * v + 256);
  }
};

// X = U^-1 L^-1 B[perm]; X may alias B.
int solve_impl(const double* LU, int64_t n, int64_t lda, const int64_t* perm, const double* Bsrc,
               int64_t ldb, double* X, int64_t nrhs, int64_t ldx, char* ws, hipStream_t st,
               const uint32_t* skip = nullptr) {
  SolveWs w(ws, n, nrhs);
  // gather B[perm] into t1, sentinel into t2, zero both tickets
  PRRP_TRY(launch_gather_rows(Bsrc, ldb, perm, w.t1, nrhs, n, nrhs, w.t2, nrhs, w.ticket, skip,
                              st));
  // L y = t1 into t2; each block then fills its rows of X with the sentinel
  // (B, which X may alias, has been read by the gather)
  PRRP_TRY(launch_trsv_blocked(LU, n, lda, w.t1, nrhs, w.t2, nrhs, nrhs, 1, w.ticket, X, ldx, skip,
                               st));
  // U x = y straight into X
  PRRP_TRY(launch_trsv_blocked(LU, n, lda, w.t2, nrhs, X, ldx, nrhs, 0, w.ticket + 1, nullptr, 0,
                               skip, st));
  return 0;
}

// Y = the forward sweep of the block factorization applied to B[perm], then
// X = U^-1 Y.
int block_solve_impl(const double* LU, int64_t n, int64_t lda, int b, const int64_t* perm,
                     const int32_t* nodes, const double* B, int64_t ldb, double* X, int64_t ldx,
                     int64_t nrhs, char* ws, hipStream_t st) {
  SolveWs w(ws, n, nrhs);
  PRRP_TRY(launch_gather_rows(B, ldb, perm, w.t1, nrhs, n, nrhs, w.t2, nrhs, w.ticket, nullptr, st));
  double* cur = w.t1;
  double* nxt = w.r;
  const int P = (int)((n + b - 1) / b);
  for (int j = 0; j < P; ++j) {
    BlockForwardArgs fa{LU, lda, n, b, j, nodes, cur, nxt, nrhs, nrhs};
    PRRP_TRY(launch_block_forward(fa, st));
    std::swap(cur, nxt);
  }
  PRRP_TRY(launch_trsv_blocked(LU, n, lda, cur, nrhs, w.t2, nrhs, nrhs, 0, w.ticket + 1, nullptr, 0,
                               nullptr, st));
  PRRP_TRY(launch_copy_rows(w.t2, nrhs, X, ldx, n, nrhs, st));
  return 0;
}
}  // namespace

int prrp_solve(const double* LU, int64_t n, int64_t lda, const int64_t* perm, double* B,
               int64_t nrhs, int64_t ldb, void* workspace, size_t ws_bytes, void* stream) {
  if (!LU) return -1;
  if (n < 1 || n > kMaxN) return -2;
  if (lda < n) return -3;
  if (!perm) return -4;
  if (!B) return -5;
  if (nrhs < 1) return -6;
  if (ldb < nrhs) return -7;
  size_t need = 0;
  prrp_solve_workspace_size(n, nrhs, &need);
  if (!workspace) return -8;
  if (ws_bytes < need) return -9;
  return solve_impl(LU, n, lda, perm, B, ldb, B, nrhs, ldb, static_cast<char*>(workspace),
                    static_cast<hipStream_t>(stream));
}

int prrp_residual(const double* A, int64_t n, int64_t lda, const double* X, const double* B,
                  double* R, int64_t nrhs, int64_t ldx, void* stream) {
  if (!A) return -1;
  if (n < 1 || n > kMaxN) return -2;
  if (lda < n) return -3;
  if (!X) return -4;
  if (!B) return -5;
  if (!R) return -6;
  if (nrhs < 1) return -7;
  if (ldx < nrhs) return -8;
  return herr(launch_residual(A, n, lda, X, ldx, B, ldx, R, ldx, nrhs, nullptr,
                              static_cast<hipStream_t>(stream)));
}

int prrp_refine(const double* A, const double* LU, int64_t n, int64_t lda, const int64_t* perm,
                const double* B, double* X, int64_t nrhs, int64_t ldx, double tol, int max_iter,
                int* iters, double* final_rel, int* status, void* workspace, size_t ws_bytes,
                void* stream) {
  if (!A) return -1;
  if (!LU) return -2;
  if (n < 1 || n > kMaxN) return -3;
  if (lda < n) return -4;
  if (!perm) return -5;
  if (!B) return -6;
  if (!X) return -7;
  if (nrhs < 1) return -8;
  if (ldx < nrhs) return -9;
  if (!(tol >= 0.0)) return -10;
  if (max_iter < 0) return -11;
  size_t need = 0;
  prrp_solve_workspace_size(n, nrhs, &need);
  if (!workspace) return -15;
  if (ws_bytes < need) return -16;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  SolveWs w(ws, n, nrhs);
  double* R = w.r;
  double* mx = w.mx;
  int rc = solve_impl(LU, n, lda, perm, B, ldx, X, nrhs, ldx, ws, st);
  if (rc) return rc;
  std::vector<double> h(2 * nrhs);
  double prev = INFINITY;
  int it = 0;
  double rel = INFINITY;
  int stat = PRRP_IR_CAP;        // the same test as the device-side loop
  for (it = 1; it <= max_iter; ++it) {
    PRRP_TRY(launch_residual(A, n, lda, X, ldx, B, ldx, R, nrhs, nrhs, nullptr, st));
    rc = solve_impl(LU, n, lda, perm, R, nrhs, R, nrhs, nrhs, ws, st);
    if (rc) return rc;
    PRRP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(mx), 2 * nrhs, 0ull, st));
    PRRP_TRY(launch_axpy_maxrel(X, ldx, R, nrhs, n, nrhs, mx, nullptr, st));
    PRRP_TRY(hipMemcpyAsync(h.data(), mx, 2 * nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    PRRP_TRY(hipStreamSynchronize(st));
    rel = 0.0;
    for (int64_t r = 0; r < nrhs; ++r) {
      const double xm = h[2 * r + 1] > 0.0 ? h[2 * r + 1] : 1.0;
      rel = std::max(rel, h[2 * r] / xm);
    }
    if (rel <= tol) { stat = PRRP_IR_CONVERGED; break; }
    if (!(rel <= 0.5 * prev)) { stat = PRRP_IR_STAGNATED; break; }
    prev = rel;
  }
  if (iters) *iters = std::min(it, max_iter);
  if (final_rel) *final_rel = max_iter > 0 ? rel : 0.0;
  if (status) *status = stat;
  return 0;
}

int prrp_refine_async(const double* A, const double* LU, int64_t n, int64_t lda,
                      const int64_t* perm, const double* B, double* X, int64_t nrhs, int64_t ldx,
                      double tol, int max_iter, int32_t* iters, double* final_rel,
                      int32_t* status, void* workspace, size_t ws_bytes, void* stream) {
  if (!A) return -1;
  if (!LU) return -2;
  if (n < 1 || n > kMaxN) return -3;
  if (lda < n) return -4;
  if (!perm) return -5;
  if (!B) return -6;
  if (!X) return -7;
  if (nrhs < 1) return -8;
  if (ldx < nrhs) return -9;
  if (!(tol >= 0.0)) return -10;
  if (max_iter < 0 || max_iter > 1000) return -11;
  size_t need = 0;
  prrp_solve_workspace_size(n, nrhs, &need);
  if (!workspace) return -15;
  if (ws_bytes < need) return -16;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  SolveWs w(ws, n, nrhs);
  PRRP_TRY(launch_ir_init(w.ir, w.mx, nrhs, iters, final_rel, status, st));
  int rc = solve_impl(LU, n, lda, perm, B, ldx, X, nrhs, ldx, ws, st);
  if (rc) return rc;
  const uint32_t* done = &w.ir->done;
  for (int it = 1; it <= max_iter; ++it) {
    PRRP_TRY(launch_residual(A, n, lda, X, ldx, B, ldx, w.r, nrhs, nrhs, done, st));
    rc = solve_impl(LU, n, lda, perm, w.r, nrhs, w.r, nrhs, nrhs, ws, st, done);
    if (rc) return rc;
    PRRP_TRY(launch_axpy_maxrel(X, ldx, w.r, nrhs, n, nrhs, w.mx, done, st));
    PRRP_TRY(launch_ir_check(w.ir, w.mx, nrhs, tol, max_iter, iters, final_rel, status, st));
  }
  return 0;
}


}  // extern "C"

// ------------------------------------------ refinement without allocation
// Scratch of the entry point below: a file-scope device array, one copy per
// GPU, held until the process ends.  Host code never passes the array's name
// to a kernel or copy (on the host it is a stand-in, not a device address):
// each device's address comes from hipGetSymbolAddress, taken once with that
// device current.
namespace {
constexpr size_t kStaticScratchBytes = (size_t)16 << 20;
}
static __device__ __align__(256) char scratch[kStaticScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}
}  // namespace

extern "C" {

size_t prrp_static_scratch_bytes(void) { return kStaticScratchBytes; }

int prrp_refine_async_static(const double* A, const double* LU, int64_t n, int64_t lda,
                             const int64_t* perm, const double* B, double* X, int64_t nrhs,
                             int64_t ldx, double tol, int max_iter, int32_t* iters,
                             double* final_rel, int32_t* status, void* stream) {
  if (n < 1 || n > kMaxN) return -3;
  if (nrhs < 1) return -8;
  size_t need = 0;
  prrp_solve_workspace_size(n, nrhs, &need);
  if (need > kStaticScratchBytes) return -8;     // n x nrhs beyond the static scratch
  void* ws = nullptr;
  const hipError_t e = scratch_address(&ws);
  if (e != hipSuccess) return herr(e);
  return prrp_refine_async(A, LU, n, lda, perm, B, X, nrhs, ldx, tol, max_iter, iters, final_rel,
                           status, ws, kStaticScratchBytes, stream);
}

}  // extern "C"

extern "C" {

// ------------------------------------------------ GMRES-based refinement
namespace {
constexpr int kGmresMax = 128;     // Krylov vectors per correction
struct GmresWs {
  double *V, *t, *z, *zero, *part, *small;
  // small: c[128] | c2[128] | y[128] | hn | beta | w | minus_one
  double* c() { return small; }
  double* c2() { return small + kGmresMax; }
  double* y() { return small + 2 * kGmresMax; }
  double* hn() { return small + 3 * kGmresMax; }
  double* beta() { return small + 3 * kGmresMax + 1; }
  double* w() { return small + 3 * kGmresMax + 2; }
  double* minus_one() { return small + 3 * kGmresMax + 3; }
};
size_t gmres_extra_bytes(int64_t n, int max_inner) {
  return align_up((size_t)(max_inner + 1) * n * 8, 256) + 3 * align_up((size_t)n * 8, 256) +
         align_up((size_t)256 * kGmresMax * 8, 256) + align_up((size_t)(3 * kGmresMax + 8) * 8, 256);
}
GmresWs gmres_ws(char* base, int64_t n, int max_inner) {
  GmresWs g;
  size_t off = 0;
  auto take = [&](size_t bytes) { char* p = base + off; off += align_up(bytes, 256); return p; };
  g.V = reinterpret_cast<double*>(take((size_t)(max_inner + 1) * n * 8));
  g.t = reinterpret_cast<double*>(take((size_t)n * 8));
  g.z = reinterpret_cast<double*>(take((size_t)n * 8));
  g.zero = reinterpret_cast<double*>(take((size_t)n * 8));
  g.part = reinterpret_cast<double*>(take((size_t)256 * kGmresMax * 8));
  g.small = reinterpret_cast<double*>(take((size_t)(3 * kGmresMax + 8) * 8));
  return g;
}
uint64_t dbits(double v) { uint64_t u; std::memcpy(&u, &v, 8); return u; }
}  // namespace

int prrp_gmres_workspace_size(int64_t n, int max_inner, size_t* bytes) {
  if (n < 1 || n > kMaxN) return -1;
  if (max_inner < 1 || max_inner > kGmresMax) return -2;
  if (!bytes) return -3;
  size_t sws = 0;
  prrp_solve_workspace_size(n, 1, &sws);
  *bytes = align_up(sws, 256) + gmres_extra_bytes(n, max_inner);
  return 0;
}

int prrp_refine_gmres(const double* A, const double* LU, int64_t n, int64_t lda,
                      const int64_t* perm, const double* b, double* x, double tol,
                      double gmres_tol, int max_inner, int max_outer, int* outer, int* inner,
                      double* w_before, double* w_final, double* final_rel, int* status,
                      void* workspace, size_t ws_bytes, void* stream) {
  if (!A) return -1;
  if (!LU) return -2;
  if (n < 1 || n > kMaxN) return -3;
  if (lda < n) return -4;
  if (!perm) return -5;
  if (!b) return -6;
  if (!x) return -7;
  if (!(tol >= 0.0)) return -8;
  if (!(gmres_tol >= 0.0) || !(gmres_tol < 1.0)) return -9;
  if (max_inner < 1 || max_inner > kGmresMax) return -10;
  if (max_outer < 0) return -11;
  size_t need = 0;
  prrp_gmres_workspace_size(n, max_inner, &need);
  if (!workspace) return -18;
  if (ws_bytes < need) return -19;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* ws = static_cast<char*>(workspace);
  size_t sws = 0;
  prrp_solve_workspace_size(n, 1, &sws);
  char* sw = ws;
  GmresWs g = gmres_ws(ws + align_up(sws, 256), n, max_inner);
  SolveWs w(sw, n, 1);
  const double u = std::ldexp(1.0, -53);
  PRRP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(g.zero), (size_t)n, 0ull, st));
  PRRP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(g.minus_one()), 1, dbits(-1.0), st));
  // x0 = U^-1 L^-1 b[perm]; r = b - A x0 and w (equation "comp")
  int rc = solve_impl(LU, n, lda, perm, b, 1, x, 1, 1, sw, st);
  if (rc) return rc;
  auto residual_w = [&](double* wh) -> int {
    PRRP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(g.w()), 1, 0ull, st));
    PRRP_TRY(launch_residual_w(A, n, lda, x, 1, b, 1, w.r, 1, 1, g.w(), st));
    PRRP_TRY(hipMemcpyAsync(wh, g.w(), 8, hipMemcpyDeviceToHost, st));
    PRRP_TRY(hipStreamSynchronize(st));
    return 0;
  };
  double wcur = 0.0;
  if ((rc = residual_w(&wcur))) return rc;
  if (w_before) *w_before = wcur;
  int stat = (tol == 0.0 && wcur <= u) ? PRRP_IR_CONVERGED : PRRP_IR_CAP;
  int steps = 0, total_inner = 0;
  double prev_rel = INFINITY, rel = INFINITY;
  std::vector<double> H((size_t)(kGmresMax + 1) * kGmresMax, 0.0), cs(kGmresMax), sn(kGmresMax),
      gv(kGmresMax + 1), hbuf(2 * kGmresMax + 4), yv(kGmresMax);
  while (stat == PRRP_IR_CAP && steps < max_outer) {
    // GMRES on U^-1 L^-1 A d = U^-1 L^-1 r (Carson and Higham, 2018)
    rc = solve_impl(LU, n, lda, perm, w.r, 1, g.z, 1, 1, sw, st);
    if (rc) return rc;
    PRRP_TRY(launch_nrm2(g.z, n, g.part, g.beta(), st));
    double beta = 0.0;
    PRRP_TRY(hipMemcpyAsync(&beta, g.beta(), 8, hipMemcpyDeviceToHost, st));
    PRRP_TRY(hipStreamSynchronize(st));
    if (!(beta > 0.0) || !std::isfinite(beta)) { stat = PRRP_IR_STAGNATED; break; }
    PRRP_TRY(launch_combine(g.V, n, 0, nullptr, 0.0, g.z, g.beta(), g.V, st));
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int k = 0;
    for (int j = 0; j < max_inner; ++j) {
      double* Vj = g.V + (size_t)j * n;
      double* Vn = g.V + (size_t)(j + 1) * n;
      // t = -A V_j; q = U^-1 L^-1 t[perm]; w = -q
      PRRP_TRY(launch_residual(A, n, lda, Vj, 1, g.zero, 1, g.t, 1, 1, nullptr, st));
      rc = solve_impl(LU, n, lda, perm, g.t, 1, g.t, 1, 1, sw, st);
      if (rc) return rc;
      PRRP_TRY(launch_combine(g.V, n, 0, nullptr, 0.0, g.t, g.minus_one(), nullptr, st));
      // classical Gram-Schmidt, twice
      PRRP_TRY(launch_dots(g.V, n, j + 1, g.t, g.part, g.c(), 0, st));
      PRRP_TRY(launch_combine(g.V, n, j + 1, g.c(), -1.0, g.t, nullptr, nullptr, st));
      PRRP_TRY(launch_dots(g.V, n, j + 1, g.t, g.part, g.c2(), 0, st));
      PRRP_TRY(launch_combine(g.V, n, j + 1, g.c2(), -1.0, g.t, nullptr, nullptr, st));
      PRRP_TRY(launch_nrm2(g.t, n, g.part, g.hn(), st));
      PRRP_TRY(launch_combine(g.V, n, 0, nullptr, 0.0, g.t, g.hn(), Vn, st));
      PRRP_TRY(hipMemcpyAsync(hbuf.data(), g.small, (2 * kGmresMax) * 8, hipMemcpyDeviceToHost, st));
      PRRP_TRY(hipMemcpyAsync(hbuf.data() + 2 * kGmresMax, g.hn(), 8, hipMemcpyDeviceToHost, st));
      PRRP_TRY(hipStreamSynchronize(st));
      double* Hj = H.data() + (size_t)j;                 // column j, row stride kGmresMax
      for (int i = 0; i <= j; ++i) Hj[(size_t)i * kGmresMax] = hbuf[i] + hbuf[kGmresMax + i];
      Hj[(size_t)(j + 1) * kGmresMax] = hbuf[2 * kGmresMax];
      for (int i = 0; i < j; ++i) {                      // earlier rotations
        const double a0 = Hj[(size_t)i * kGmresMax], a1 = Hj[(size_t)(i + 1) * kGmresMax];
        Hj[(size_t)i * kGmresMax] = cs[i] * a0 + sn[i] * a1;
        Hj[(size_t)(i + 1) * kGmresMax] = -sn[i] * a0 + cs[i] * a1;
      }
      const double a0 = Hj[(size_t)j * kGmresMax], a1 = Hj[(size_t)(j + 1) * kGmresMax];
      const double hyp = std::hypot(a0, a1);
      cs[j] = hyp > 0.0 ? a0 / hyp : 1.0;
      sn[j] = hyp > 0.0 ? a1 / hyp : 0.0;
      Hj[(size_t)j * kGmresMax] = hyp;
      Hj[(size_t)(j + 1) * kGmresMax] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      k = j + 1;
      if (std::fabs(gv[j + 1]) <= gmres_tol * beta || hyp == 0.0) break;
    }
    total_inner += k;
    for (int i = k - 1; i >= 0; --i) {
      double acc = gv[i];
      for (int c = i + 1; c < k; ++c) acc -= H[(size_t)i * kGmresMax + c] * yv[c];
      const double d = H[(size_t)i * kGmresMax + i];
      yv[i] = d != 0.0 ? acc / d : 0.0;
    }
    PRRP_TRY(hipMemcpyAsync(g.y(), yv.data(), (size_t)k * 8, hipMemcpyHostToDevice, st));
    // d = V y into t; x += d with max|d| and max|x| (the correction's size)
    PRRP_TRY(launch_combine(g.V, n, k, g.y(), 1.0, nullptr, nullptr, g.t, st));
    PRRP_TRY(launch_fill_u64(reinterpret_cast<uint64_t*>(g.c2()), 2, 0ull, st));
    PRRP_TRY(launch_axpy_maxrel(x, 1, g.t, 1, n, 1, g.c2(), nullptr, st));
    double mx[2] = {0.0, 0.0};
    PRRP_TRY(hipMemcpyAsync(mx, g.c2(), 16, hipMemcpyDeviceToHost, st));
    ++steps;
    double wnew = 0.0;
    if ((rc = residual_w(&wnew))) return rc;           // synchronizes: mx is in
    rel = mx[0] / (mx[1] > 0.0 ? mx[1] : 1.0);
    if (tol > 0.0) {
      if (rel <= tol) stat = PRRP_IR_CONVERGED;
      else if (!(rel <= 0.5 * prev_rel)) stat = PRRP_IR_STAGNATED;
      prev_rel = rel;
    } else if (wnew <= u) {
      stat = PRRP_IR_CONVERGED;
    } else if (!(wnew <= 0.5 * wcur)) {
      stat = PRRP_IR_STAGNATED;
    }
    wcur = wnew;
  }
  if (outer) *outer = steps;
  if (inner) *inner = total_inner;
  if (w_final) *w_final = wcur;
  if (final_rel) *final_rel = steps > 0 ? rel : 0.0;
  if (status) *status = stat;
  return 0;
}

}  // extern "C"

// ==========================================================================
// Batched factorization of many independent systems (uneven sizes).
//
// A plan fixes the problems (pointers and sizes) and precomputes, for every
// panel step, one work list per kernel: the strong-RRQR launch of a step
// covers every problem still active (one group of workgroups per problem,
// problems of equal panel width and workgroup count sharing a launch), and
// the diagonal GEPP, row moves, L21 product, U12 solve and Schur update of
// the step are one launch each over all active problems.  Its device memory
// (work lists and per-problem workspaces) is a caller-provided workspace.
// The launch sequence can be captured once into a HIP graph and replayed;
// optional refinement of every system runs as one launch per sub-step over
// the whole batch.
// ==========================================================================
namespace {

struct PlanProblem {
  double* A;
  int64_t n, lda;
  int b;
  int64_t* perm;
  prrp_stats* stats;
  int Gmax;
  size_t set_words;
  size_t off_slots, off_rounds, off_sel, off_y, off_pl, off_mv, off_sws, off_p11;
  // refinement (A0 == nullptr: none)
  const double* A0;
  const double* B;
  double* X;
  int64_t nrhs;
  char* sws;
  size_t sws_bytes;
};

enum OpKind { OP_SRRQR = 0, OP_PLAN, OP_MOVES, OP_SCHUR, OP_GEPP, OP_PERMTOP, OP_L21, OP_U12 };
struct PlanOp {
  OpKind kind;
  size_t off;          // byte offset of the work list in the workspace
  int count;
  int bw;
  int64_t max_a, max_b;
  int prec;
  int srrqr_index;     // OP_SRRQR: index into srrqr_args
};

struct BatchPlan {
  double tau = 2.0;
  int schur = 0;
  int rpw_target = 64;
  double tol = 0.0;
  int max_iter = 0;
  bool refine = false;
  std::vector<PlanProblem> p;
  char* base = nullptr;             // workspace
  size_t need = 0;
  size_t lists_at = 0;
  size_t slots_begin = 0, slots_end = 0;
  size_t off_abort = 0, off_iters = 0, off_rels = 0, off_status = 0;
  std::vector<char> host;           // work lists (host image, uploaded at creation)
  std::vector<PlanOp> ops;
  std::vector<SrrqrArgs> srrqr_args;
  std::vector<size_t> srrqr_list_off;
  size_t ir_list_off = 0;           // refinement work list (relative to lists_at)
  int64_t max_n = 0, max_nrhs = 0;
  hipStream_t cap = nullptr;        // private stream the graph is captured on
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Lays out the workspace and builds every step's work lists (offsets stand in
// for device pointers until relocate(); no offset is 0, which means "none").
void plan_build(BatchPlan& P) {
  const int cap = std::min(256, device_cus());
  const int64_t count = (int64_t)P.p.size();
  size_t off = 256;
  auto take = [&](size_t bytes) { size_t o = off; off += align_up(bytes, 256); return o; };
  P.slots_begin = off;
  for (auto& q : P.p) {
    q.Gmax = groups_for_rows(q.n, cap, 64, q.b);
    q.set_words = (size_t)q.Gmax * kRoundsMax * kPostW;
    q.off_slots = take(2 * q.set_words * 8);
  }
  P.slots_end = off;
  for (auto& q : P.p) {
    q.off_rounds = take(2 * 4);
    q.off_sel = take(kMaxB * 4);
    q.off_y = take((size_t)q.n * q.b * 8);
    q.off_pl = take((size_t)q.b * q.b * 8);
    q.off_mv = take((4 * kMaxB + 4) * 4);
    q.off_p11 = take(kMaxB * 4);
    q.off_sws = 0;
    if (P.refine) {
      prrp_solve_workspace_size(q.n, q.nrhs, &q.sws_bytes);
      q.off_sws = take(q.sws_bytes);
    }
  }
  P.off_abort = take(256);
  P.off_iters = take((size_t)count * 4);
  P.off_rels = take((size_t)count * 8);
  P.off_status = take((size_t)count * 4);
  P.lists_at = align_up(off, 256);

  std::vector<char>& host = P.host;
  host.clear();
  auto put = [&](const void* src, size_t bytes) {
    const size_t o = align_up(host.size(), 256);
    host.resize(o + bytes);
    std::memcpy(host.data() + o, src, bytes);
    return o;
  };
  auto W = [](size_t o) { return reinterpret_cast<char*>(o); };   // offset as pointer
  std::vector<int> prevG(count, 0), prevBw(count, 0);
  int64_t steps = 0;
  for (auto& q : P.p) steps = std::max<int64_t>(steps, (q.n + q.b - 1) / q.b);
  for (int64_t s = 0; s < steps; ++s) {
    const int par = (int)(s & 1);
    std::vector<std::pair<std::pair<int, int>, int>> cls;   // ((bw, G), problem)
    for (int64_t i = 0; i < count; ++i) {
      const PlanProblem& q = P.p[i];
      const int64_t k0 = s * q.b;
      if (k0 >= q.n) continue;
      const int64_t m = q.n - k0;
      const int bw = (int)std::min<int64_t>(q.b, m);
      cls.push_back({{bw, groups_for_rows(m, cap, P.rpw_target, bw)}, (int)i});
    }
    std::stable_sort(cls.begin(), cls.end(),
                     [](const auto& x, const auto& y) { return x.first < y.first; });
    for (size_t c0 = 0; c0 < cls.size();) {
      size_t c1 = c0;
      while (c1 < cls.size() && cls[c1].first == cls[c0].first) ++c1;
      const int bw = cls[c0].first.first, G = cls[c0].first.second;
      std::vector<SrrqrProblem> list;
      int64_t maxm = 0;
      for (size_t c = c0; c < c1; ++c) {
        const int i = cls[c].second;
        const PlanProblem& q = P.p[i];
        const int64_t k0 = s * q.b, m = q.n - k0;
        maxm = std::max(maxm, m);
        SrrqrProblem sp;
        std::memset(&sp, 0, sizeof sp);
        sp.A = q.A; sp.lda = q.lda; sp.k0 = k0; sp.m = (int)m;
        sp.Y = (m > bw) ? reinterpret_cast<double*>(W(q.off_y)) : nullptr;
        sp.ldy = q.b;
        sp.sel_out = reinterpret_cast<int32_t*>(W(q.off_sel));
        sp.slots = reinterpret_cast<uint64_t*>(W(q.off_slots + (size_t)par * q.set_words * 8));
        sp.rounds_out = reinterpret_cast<int32_t*>(W(q.off_rounds + (size_t)par * 4));
        if (s > 0) {
          sp.clear_base = reinterpret_cast<uint64_t*>(W(q.off_slots + (size_t)(1 - par) * q.set_words * 8));
          sp.clear_G = prevG[i];
          sp.clear_bw = prevBw[i];
          sp.clear_rounds = reinterpret_cast<int32_t*>(W(q.off_rounds + (size_t)(1 - par) * 4));
        }
        sp.stats = q.stats;
        list.push_back(sp);
        prevG[i] = G;
        prevBw[i] = bw;
      }
      SrrqrArgs a;
      std::memset(&a, 0, sizeof a);
      a.bw = bw;
      a.ngroups = (int)list.size();
      a.G = G;
      a.rpw = (int)((maxm + G - 1) / G);
      a.tau_bits = tau_bits(P.tau);
      a.report_rank = 1;
      a.record_block_L = 1;
      const size_t lo = put(list.data(), list.size() * sizeof(SrrqrProblem));
      P.ops.push_back(PlanOp{OP_SRRQR, lo, (int)list.size(), bw, 0, 0, 0, (int)P.srrqr_args.size()});
      P.srrqr_args.push_back(a);
      P.srrqr_list_off.push_back(lo);
      c0 = c1;
    }
    std::vector<GeppArgs> gl;
    std::vector<MoveArgs> ml;
    std::vector<GemmArgs> l21, sch;
    std::vector<TrsmArgs> tl;
    std::vector<PermTopArgs> pl;
    int maxbw = 0;
    int64_t maxout = 0, maxm2 = 0, maxnr = 0, maxk0 = 0;
    for (int64_t i = 0; i < count; ++i) {
      const PlanProblem& q = P.p[i];
      const int64_t k0 = s * q.b;
      if (k0 >= q.n) continue;
      const int64_t m = q.n - k0;
      const int bw = (int)std::min<int64_t>(q.b, m);
      maxbw = std::max(maxbw, bw);
      maxk0 = std::max(maxk0, k0);
      int32_t* mv_dst = reinterpret_cast<int32_t*>(W(q.off_mv));
      int32_t* mv_src = reinterpret_cast<int32_t*>(W(q.off_mv + 2 * kMaxB * 4));
      int32_t* n_moves = reinterpret_cast<int32_t*>(W(q.off_mv + 4 * kMaxB * 4));
      int32_t* p11 = reinterpret_cast<int32_t*>(W(q.off_p11));
      double* Yp = reinterpret_cast<double*>(W(q.off_y));
      double* PLp = reinterpret_cast<double*>(W(q.off_pl));
      gl.push_back(GeppArgs{q.A, q.lda, k0, bw, (int)m, reinterpret_cast<int32_t*>(W(q.off_sel)),
                            PLp, mv_dst, mv_src, n_moves, q.stats, p11});
      ml.push_back(MoveArgs{q.A, q.lda, q.n, k0, bw, mv_dst, mv_src, n_moves, q.perm,
                            (m > bw) ? Yp : nullptr, q.b, 0, q.n, k0, bw});
      pl.push_back(PermTopArgs{q.A, q.lda, k0, bw, q.perm, p11});
      maxout = std::max<int64_t>(maxout, q.n - bw);
      if (m > bw) {
        const int64_t nr = q.n - k0 - bw;
        // M^T rows from bw on: offset of Y plus bw rows of ld b
        double* Yrows = reinterpret_cast<double*>(W(q.off_y + (size_t)bw * q.b * 8));
        // block form A22 -= M^T A12 (A12 before the diagonal GEPP)
        sch.push_back(GemmArgs{(int)(m - bw), (int)nr, bw, Yrows, q.b,
                               q.A + k0 * q.lda + k0 + bw, q.lda, q.A + (k0 + bw) * q.lda + k0 + bw,
                               q.lda, -1.0, 1.0, &q.stats->max_abs_W, nullptr, P.schur});
        l21.push_back(GemmArgs{(int)(m - bw), bw, bw, Yrows, q.b, PLp, bw,
                               q.A + (k0 + bw) * q.lda + k0, q.lda, 1.0, 0.0, nullptr, nullptr,
                               PRRP_FP64});
        tl.push_back(TrsmArgs{q.A, q.lda, k0, bw, nr, &q.stats->max_abs_U, &q.stats->max_abs_W,
                              p11});
        maxm2 = std::max<int64_t>(maxm2, m - bw);
        maxnr = std::max<int64_t>(maxnr, nr);
      }
    }
    P.ops.push_back(PlanOp{OP_PLAN, put(gl.data(), gl.size() * sizeof(GeppArgs)), (int)gl.size(),
                           maxbw, 0, 0, 0, -1});
    P.ops.push_back(PlanOp{OP_MOVES, put(ml.data(), ml.size() * sizeof(MoveArgs)), (int)ml.size(),
                           maxbw, maxout, 0, 0, -1});
    if (!sch.empty())
      P.ops.push_back(PlanOp{OP_SCHUR, put(sch.data(), sch.size() * sizeof(GemmArgs)),
                             (int)sch.size(), maxbw, maxm2, maxnr, P.schur, -1});
    P.ops.push_back(PlanOp{OP_GEPP, put(gl.data(), gl.size() * sizeof(GeppArgs)), (int)gl.size(),
                           maxbw, 0, 0, 0, -1});
    P.ops.push_back(PlanOp{OP_PERMTOP, put(pl.data(), pl.size() * sizeof(PermTopArgs)),
                           (int)pl.size(), maxbw, maxk0, 0, 0, -1});
    if (!l21.empty()) {
      P.ops.push_back(PlanOp{OP_L21, put(l21.data(), l21.size() * sizeof(GemmArgs)),
                             (int)l21.size(), maxbw, maxm2, maxbw, PRRP_FP64, -1});
      P.ops.push_back(PlanOp{OP_U12, put(tl.data(), tl.size() * sizeof(TrsmArgs)), (int)tl.size(),
                             maxbw, maxnr, 0, 0, -1});
    }
  }
  if (P.refine) {
    std::vector<IrArgs> irl(count);
    std::memset(irl.data(), 0, irl.size() * sizeof(IrArgs));
    P.ir_list_off = put(irl.data(), irl.size() * sizeof(IrArgs));
    for (auto& q : P.p) {
      P.max_n = std::max(P.max_n, q.n);
      P.max_nrhs = std::max(P.max_nrhs, q.nrhs);
    }
  }
  P.need = P.lists_at + host.size();
}

// Turns the offsets in the work lists into addresses in the workspace.
void plan_relocate(BatchPlan& P) {
  char* base = P.base;
  auto R = [&](auto*& ptr) {
    if (ptr != nullptr)
      ptr = reinterpret_cast<std::remove_reference_t<decltype(ptr)>>(
          base + reinterpret_cast<size_t>(ptr));
  };
  for (size_t k = 0; k < P.srrqr_args.size(); ++k) {
    SrrqrProblem* lst = reinterpret_cast<SrrqrProblem*>(P.host.data() + P.srrqr_list_off[k]);
    for (int g = 0; g < P.srrqr_args[k].ngroups; ++g) {
      SrrqrProblem& sp = lst[g];
      R(sp.Y); R(sp.sel_out); R(sp.slots); R(sp.rounds_out); R(sp.clear_base); R(sp.clear_rounds);
    }
    P.srrqr_args[k].probs =
        reinterpret_cast<const SrrqrProblem*>(base + P.lists_at + P.srrqr_list_off[k]);
    P.srrqr_args[k].abort_flag = reinterpret_cast<uint32_t*>(base + P.off_abort);
  }
  for (PlanOp& o : P.ops) {
    char* h = P.host.data() + o.off;
    if (o.kind == OP_GEPP || o.kind == OP_PLAN) {
      GeppArgs* g = reinterpret_cast<GeppArgs*>(h);
      for (int k = 0; k < o.count; ++k) {
        R(g[k].sel); R(g[k].PL); R(g[k].mv_dst); R(g[k].mv_src); R(g[k].n_moves); R(g[k].p11);
      }
    } else if (o.kind == OP_MOVES) {
      MoveArgs* m = reinterpret_cast<MoveArgs*>(h);
      for (int k = 0; k < o.count; ++k) { R(m[k].mv_dst); R(m[k].mv_src); R(m[k].n_moves); R(m[k].Y); }
    } else if (o.kind == OP_L21) {
      GemmArgs* g = reinterpret_cast<GemmArgs*>(h);
      for (int k = 0; k < o.count; ++k) { R(g[k].A); R(g[k].B); }
    } else if (o.kind == OP_SCHUR) {
      GemmArgs* g = reinterpret_cast<GemmArgs*>(h);
      for (int k = 0; k < o.count; ++k) R(g[k].A);
    } else if (o.kind == OP_PERMTOP) {
      PermTopArgs* t = reinterpret_cast<PermTopArgs*>(h);
      for (int k = 0; k < o.count; ++k) R(t[k].p11);
    } else if (o.kind == OP_U12) {
      TrsmArgs* t = reinterpret_cast<TrsmArgs*>(h);
      for (int k = 0; k < o.count; ++k) R(t[k].p11);
    }
    o.off += P.lists_at;
  }
  if (P.refine) {
    IrArgs* irl = reinterpret_cast<IrArgs*>(P.host.data() + P.ir_list_off);
    int32_t* iters = reinterpret_cast<int32_t*>(base + P.off_iters);
    double* rels = reinterpret_cast<double*>(base + P.off_rels);
    int32_t* stat = reinterpret_cast<int32_t*>(base + P.off_status);
    for (size_t i = 0; i < P.p.size(); ++i) {
      PlanProblem& q = P.p[i];
      q.sws = base + q.off_sws;
      SolveWs w(q.sws, q.n, q.nrhs);
      irl[i] = IrArgs{q.A0, q.n, q.lda, q.A, q.perm, q.B, q.X, q.nrhs, w.t1, w.t2, w.r, w.mx,
                      w.ticket, w.ir, iters + i, rels + i, stat + i};
    }
  }
}

hipError_t plan_enqueue(BatchPlan& P, hipStream_t st) {
  hipError_t e;
  uint32_t* abort_flag = reinterpret_cast<uint32_t*>(P.base + P.off_abort);
  for (auto& q : P.p) {
    e = launch_init_factor(q.A, q.n, q.lda, q.perm, q.stats, abort_flag, 0,
                           (int)((q.n + q.b - 1) / q.b), st);
    if (e != hipSuccess) return e;
  }
  e = launch_fill_u64(reinterpret_cast<uint64_t*>(P.base + P.slots_begin),
                      (P.slots_end - P.slots_begin) / 8, kKeySent, st);
  if (e != hipSuccess) return e;
  for (const PlanOp& o : P.ops) {
    char* list = P.base + o.off;
    switch (o.kind) {
      case OP_SRRQR: e = launch_srrqr(P.srrqr_args[o.srrqr_index], st); break;
      case OP_PLAN: e = launch_plan_batched(reinterpret_cast<GeppArgs*>(list), o.count, st); break;
      case OP_GEPP: e = launch_gepp_batched(reinterpret_cast<GeppArgs*>(list), o.count, o.bw, st); break;
      case OP_PERMTOP:
        e = launch_perm_top_batched(reinterpret_cast<PermTopArgs*>(list), o.count, o.max_a, st);
        break;
      case OP_MOVES:
        e = launch_moves_batched(reinterpret_cast<MoveArgs*>(list), o.count, o.max_a, st);
        break;
      case OP_L21:
      case OP_SCHUR:
        e = launch_gemm_batched(reinterpret_cast<GemmArgs*>(list), o.count, (int)o.max_a,
                                (int)o.max_b, o.prec, st);
        break;
      case OP_U12:
        e = launch_trsm_u12_batched(reinterpret_cast<TrsmArgs*>(list), o.count, o.bw, o.max_a, st);
        break;
    }
    if (e != hipSuccess) return e;
  }
  if (P.refine) {
    e = launch_refine_batched(reinterpret_cast<const IrArgs*>(P.base + P.lists_at + P.ir_list_off),
                              (int)P.p.size(), P.max_n, P.max_nrhs, P.tol, P.max_iter, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

void plan_free(BatchPlan* P) {
  if (!P) return;
  if (P->exec) (void)hipGraphExecDestroy(P->exec);
  if (P->graph) (void)hipGraphDestroy(P->graph);
  if (P->cap) (void)hipStreamDestroy(P->cap);
  delete P;
}

int plan_setup(BatchPlan& P, int64_t count, double* const* A, const int64_t* n,
               const int64_t* lda, const int* b, int64_t* const* perm, prrp_stats* stats,
               double tau, int schur, int rows_per_wg, const double* const* A0,
               const double* const* B, double* const* X, const int64_t* nrhs, double tol,
               int max_iter) {
  if (count < 1 || count > 4096) return -1;
  if (!A) return -2;
  if (!n) return -3;
  if (!lda) return -4;
  if (!b) return -5;
  if (!perm) return -6;
  if (!stats) return -7;
  if (!(tau > 1.0) || !std::isfinite(tau)) return -8;
  if (schur < 0 || schur > 2) return -9;
  if (rows_per_wg != 64 && rows_per_wg != 128) return -10;
  const bool refine = A0 != nullptr;
  if (refine && (!B || !X || !nrhs)) return -11;
  if (refine && (!(tol >= 0.0) || max_iter < 0 || max_iter > 1000)) return -15;
  for (int64_t i = 0; i < count; ++i) {
    if (!A[i] || !perm[i]) return -2;
    if (n[i] < 1 || n[i] > kMaxN) return -3;
    if (lda[i] < n[i]) return -4;
    if (b[i] < 1 || b[i] > kMaxB || b[i] > n[i]) return -5;
    if (refine && (!A0[i] || !B[i] || !X[i] || nrhs[i] < 1)) return -11;
  }
  P.tau = tau;
  P.schur = schur;
  P.rpw_target = rows_per_wg;
  P.refine = refine;
  P.tol = tol;
  P.max_iter = max_iter;
  P.p.resize(count);
  for (int64_t i = 0; i < count; ++i) {
    PlanProblem& q = P.p[i];
    std::memset(&q, 0, sizeof q);
    q.A = A[i]; q.n = n[i]; q.lda = lda[i]; q.b = b[i]; q.perm = perm[i]; q.stats = stats + i;
    if (refine) { q.A0 = A0[i]; q.B = B[i]; q.X = X[i]; q.nrhs = nrhs[i]; }
  }
  plan_build(P);
  return 0;
}

}  // namespace

extern "C" {

int prrp_batch_plan_workspace_size(int64_t count, const int64_t* n, const int* b,
                                   const int64_t* nrhs, int rows_per_wg, size_t* bytes) {
  if (count < 1 || count > 4096) return -1;
  if (!n) return -2;
  if (!b) return -3;
  if (rows_per_wg != 64 && rows_per_wg != 128) return -5;
  if (!bytes) return -6;
  std::vector<double*> fakeA(count, reinterpret_cast<double*>(8));
  std::vector<int64_t*> fakeP(count, reinterpret_cast<int64_t*>(8));
  std::vector<const double*> fakeA0(count, reinterpret_cast<const double*>(8));
  std::vector<double*> fakeX(count, reinterpret_cast<double*>(8));
  std::vector<int64_t> lda(n, n + count);
  BatchPlan P;
  const int rc = plan_setup(P, count, fakeA.data(), n, lda.data(), b, fakeP.data(),
                            reinterpret_cast<prrp_stats*>(8), 2.0, 0, rows_per_wg,
                            nrhs ? fakeA0.data() : nullptr, nrhs ? fakeA0.data() : nullptr,
                            nrhs ? fakeX.data() : nullptr, nrhs, 0.0, 1);
  if (rc == -3 || rc == -4) return -2;
  if (rc == -5) return -3;
  if (rc == -11) return -4;
  if (rc) return rc;
  *bytes = P.need;
  return 0;
}

int prrp_batch_plan_create(int64_t count, double* const* A, const int64_t* n, const int64_t* lda,
                           const int* b, int64_t* const* perm, prrp_stats* stats, double tau,
                           int schur, int rows_per_wg, const double* const* A0,
                           const double* const* B, double* const* X, const int64_t* nrhs,
                           double tol, int max_iter, void* workspace, size_t ws_bytes,
                           void* stream, void** plan_out) {
  if (!plan_out) return -20;
  BatchPlan* P = new BatchPlan();
  int rc = plan_setup(*P, count, A, n, lda, b, perm, stats, tau, schur, rows_per_wg, A0, B, X,
                      nrhs, tol, max_iter);
  if (rc) { plan_free(P); return rc; }
  if (!workspace) { plan_free(P); return -17; }
  if (ws_bytes < P->need) { plan_free(P); return -18; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = srrqr_prepare();
  if (e == hipSuccess) e = prepare_batched_kernels();
  if (e != hipSuccess) { plan_free(P); return herr(e); }
  // each problem's strong-RRQR workgroups wait on each other: a problem
  // whose panel the device cannot hold at once is an argument error
  for (const SrrqrArgs& a : P->srrqr_args) {
    const int64_t c = tile_cus(a.G, a.bw, a.rpw);
    if (c < 0) { plan_free(P); return herr(hipErrorInvalidValue); }
    if (c > device_cus()) { plan_free(P); return -3; }
  }
  P->base = static_cast<char*>(workspace);
  plan_relocate(*P);
  // the host image stays alive in the plan until destruction
  e = hipMemcpyAsync(P->base + P->lists_at, P->host.data(), P->host.size(),
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) { plan_free(P); return herr(e); }
  *plan_out = P;
  return 0;
}

int prrp_batch_plan_run(void* plan, void* stream, int use_graph) {
  if (!plan) return -1;
  BatchPlan& P = *static_cast<BatchPlan*>(plan);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (!use_graph) return herr(plan_enqueue(P, st));
  if (!P.exec) {
    // captured on a private stream (the caller's may be the legacy default
    // stream, which cannot be captured); the graph is launched on the caller's
    if (!P.cap) PRRP_TRY(hipStreamCreateWithFlags(&P.cap, hipStreamNonBlocking));
    PRRP_TRY(hipStreamBeginCapture(P.cap, hipStreamCaptureModeRelaxed));
    const hipError_t e = plan_enqueue(P, P.cap);
    hipGraph_t g = nullptr;
    const hipError_t e2 = hipStreamEndCapture(P.cap, &g);
    if (e != hipSuccess) { if (g) (void)hipGraphDestroy(g); return herr(e); }
    if (e2 != hipSuccess) return herr(e2);
    P.graph = g;
    PRRP_TRY(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
  }
  return herr(hipGraphLaunch(P.exec, st));
}

int prrp_batch_plan_results(void* plan, int32_t* iters, double* rels, int32_t* status,
                            void* stream) {
  if (!plan) return -1;
  BatchPlan& P = *static_cast<BatchPlan*>(plan);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t c = P.p.size();
  if (iters) PRRP_TRY(hipMemcpyAsync(iters, P.base + P.off_iters, c * 4, hipMemcpyDeviceToHost, st));
  if (rels) PRRP_TRY(hipMemcpyAsync(rels, P.base + P.off_rels, c * 8, hipMemcpyDeviceToHost, st));
  if (status)
    PRRP_TRY(hipMemcpyAsync(status, P.base + P.off_status, c * 4, hipMemcpyDeviceToHost, st));
  PRRP_TRY(hipStreamSynchronize(st));
  return 0;
}

int prrp_batch_plan_destroy(void* plan) {
  plan_free(static_cast<BatchPlan*>(plan));
  return 0;
}

// ------------------------------------- block parallel / block pairwise LU_PRRP
int prrp_block_sizes(int64_t n, int b, int tree, int64_t tile_rows, size_t* ws_bytes,
                     int64_t* node_entries) {
  if (n < 1 || n > kMaxN) return -1;
  if (b < 1 || b > kMaxB || b > n) return -2;
  if (tree != PRRP_TREE_BINARY && tree != PRRP_TREE_FLAT) return -3;
  if (tile_rows < b) return -4;
  if ((n + tile_rows - 1) / tile_rows > kMaxGroups) return -4;
  if (ws_bytes) *ws_bytes = make_block_layout(n, b, tree, tile_rows).total;
  if (node_entries) *node_entries = block_nodes_len(n, b, tree, tile_rows);
  return 0;
}

int prrp_block_factor(double* A, int64_t n, int64_t lda, int b, double tau, int tree,
                      int64_t tile_rows, int64_t* perm, int32_t* nodes, int64_t node_entries,
                      prrp_stats* stats, void* workspace, size_t ws_bytes, void* stream) {
  if (!A) return -1;
  if (n < 1 || n > kMaxN) return -2;
  if (lda < n) return -3;
  if (b < 1 || b > kMaxB || b > n) return -4;
  if (!(tau > 1.0) || !std::isfinite(tau)) return -5;
  if (tree != PRRP_TREE_BINARY && tree != PRRP_TREE_FLAT) return -6;
  if (tile_rows < b || (n + tile_rows - 1) / tile_rows > kMaxGroups) return -7;
  if (!perm) return -8;
  if (!nodes) return -9;
  if (node_entries < block_nodes_len(n, b, tree, tile_rows)) return -10;
  if (!stats) return -11;
  if (!workspace) return -12;
  if (ws_bytes < make_block_layout(n, b, tree, tile_rows).total) return -13;
  return run_block_factor(A, n, lda, b, tau, tree, tile_rows, perm, nodes, stats, workspace,
                          stream);
}

int prrp_block_solve(const double* LU, int64_t n, int64_t lda, int b, const int64_t* perm,
                     const int32_t* nodes, const double* B, int64_t ldb, double* X, int64_t ldx,
                     int64_t nrhs, void* workspace, size_t ws_bytes, void* stream) {
  if (!LU) return -1;
  if (n < 1 || n > kMaxN) return -2;
  if (lda < n) return -3;
  if (b < 1 || b > kMaxB || b > n) return -4;
  if (!perm) return -5;
  if (!nodes) return -6;
  if (!B) return -7;
  if (nrhs < 1) return -11;
  if (ldb < nrhs) return -8;
  if (!X) return -9;
  if (ldx < nrhs) return -10;
  size_t need = 0;
  prrp_solve_workspace_size(n, nrhs, &need);
  if (!workspace) return -12;
  if (ws_bytes < need) return -13;
  return block_solve_impl(LU, n, lda, b, perm, nodes, B, ldb, X, ldx, nrhs,
                          static_cast<char*>(workspace), static_cast<hipStream_t>(stream));
}

}  // extern "C"
