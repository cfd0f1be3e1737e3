// Strong rank revealing QR of a panel's transpose on gfx950.
//
// Appendix A ("Strong RRQR"): Householder QR with column pivoting of P^T,
// then interchanges while some |(R11^-1 R12)_ij| > tau.  The columns of P^T
// are the panel's rows, so a "column" here is a row of the panel.
//
// One launch handles `ngroups` independent tiles (a whole LU_PRRP panel, or the
// leaves / nodes of a CALU_PRRP tournament).  Each tile is owned by G
// workgroups; every workgroup keeps its share of the tile's rows in registers
// (8 lanes per row, lane l8 holds columns l8, l8+8, ...).  Each step of the
// pivoting needs the tile-wide winner: every workgroup posts its best
// candidate (tie key + the candidate row) into a fresh slot of device memory
// and reads the G posted keys back; slots start out holding a sentinel and
// are written exactly once, so readers simply poll until the sentinel is gone
// (device-scope atomics, no fences).  Slots alternate between two sets from
// launch to launch; a launch restores the sentinels of the set the previous
// launch used.
//
// Selection rule: QRCP recomputes the squared norm of every candidate's
// trailing part after each reflection and takes the largest under the tie
// rule (lowest tile position among equal truncated keys).  After QRCP,
// M = R11^-1 R12 is formed for every unselected row; while the largest |M|
// (tie: lowest row, then lowest slot) exceeds tau the row takes that slot and
// M is updated by the rank-one exchange formula.
#include "common.h"
#include "kernels.h"

namespace prrp {

namespace {

// Workgroup sizes: 512 threads for up to 64 rows per workgroup, 256 for up
// to 128; 1024 for a tile of up to 256 rows and at most 64 columns held by
// one workgroup.  A tile held by one workgroup never waits on device memory:
// every step's winner is found with barriers.
constexpr int kThreads = 256;
constexpr int kThreadsMid = 512;
constexpr int kThreadsWide = 1024;      // only for panels of at most 64 columns
constexpr int kRowsWide = kThreadsWide / 8 * 2;

// Poll a posted word until the sentinel is replaced; bounded.
__device__ __forceinline__ uint64_t poll_word(const uint64_t* p, const uint32_t* abort_flag,
                                              int* bad) {
  uint64_t v = ld_dev(p);
  unsigned it = 0;
  while (v == kKeySent) {
    __builtin_amdgcn_s_sleep(1);
    v = ld_dev(p);
    ++it;
    if ((it & 255u) == 0u && ld_dev_u32(abort_flag) != 0u) { *bad = 1; break; }
    if (it > kSpinLimit) { *bad = 1; break; }
  }
  return v;
}

// The largest of the keys posted at base + m * stride for this lane's slots
// m = lane, lane + 64, ... (m < G <= 256), all polled together; bounded.
// A failed wait sets *bad (the keys not yet posted then count as 0).
__device__ __forceinline__ uint64_t poll_keys(const uint64_t* base, size_t stride, int G,
                                              int lane, const uint32_t* abort_flag, int* bad) {
  uint64_t v[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int m = lane + 64 * j;
    v[j] = m < G ? ld_dev(base + (size_t)m * stride) : 0ull;
  }
  unsigned it = 0;
  for (;;) {
    bool wait = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) wait = wait || v[j] == kKeySent;
    if (!wait) break;
    ++it;
    if (((it & 255u) == 0u && ld_dev_u32(abort_flag) != 0u) || it > kSpinLimit) {
      *bad = 1;
#pragma unroll
      for (int j = 0; j < 4; ++j) v[j] = v[j] == kKeySent ? 0ull : v[j];
      break;
    }
    __builtin_amdgcn_s_sleep(1);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      if (v[j] == kKeySent) v[j] = ld_dev(base + (size_t)(lane + 64 * j) * stride);
  }
  return umax(umax(v[0], v[1]), umax(v[2], v[3]));
}

struct Smem {
  double* R;       // R11 packed by columns: R(i,j), i <= j, at j(j+1)/2 + i
  double* vsh;     // [kMaxB] reflector / exchange vector
  double* prow;    // [2 kMaxB] winner's row, zero past bw (unguarded reads)
  double* rdiag;   // [kMaxB] 1 / R(i,i)
  double* scal;    // [8]   4, 5: alpha, beta of the pivot row's reflector
  uint64_t* red;   // [2 waves + 8] reduction scratch: per-wave keys, the
                   // exchange loop's per-wave keys, the polled maximum
  int* selpos;     // [kMaxB] tile positions in slot order
  double* vw;      // [waves][2 kMaxB] per-wave reflector vectors
  int* flags;      // [8]   0: abort, 1: rank deficient, 2: winner slot,
                   //       3: exchange slot, 4: failed wait of the key poll
  int* dest;       // [kMaxB] position after Pi_j of each top-block row left out
};

}  // namespace

size_t srrqr_smem_bytes(int bw, int nt) {
  return sizeof(double) * (size_t)(bw * (bw + 1) / 2 + 4 * kMaxB + 8) +
         sizeof(double) * (size_t)(nt / 64) * 2 * kMaxB + sizeof(uint64_t) * (2 * (nt / 64) + 8) +
         sizeof(int) * (2 * kMaxB + 8);
}

// Words a post of a panel of width bw may have written: key, slot, the row
// in whole blocks of 8 columns per lane (CPT rounded as in dispatch), then
// the alpha and beta of the reflector the row defines.
__device__ __forceinline__ int post_width(int bw) {
  int cpt = (bw + 7) / 8;
  cpt = cpt <= 2 ? (cpt <= 1 ? 1 : 2) : (cpt <= 4 ? 4 : (cpt <= 8 ? 8 : 16));
  return 4 + 8 * cpt;
}

template <int CPT, int RPT, int NT>
__global__ __launch_bounds__(NT, 1)
void srrqr_kernel(SrrqrArgs a) {
  constexpr int kRowGroups = NT / 8;
  constexpr int NW = NT / 64;
  extern __shared__ double smem_raw[];
  const int bw = a.bw;
  Smem S;
  S.R = smem_raw;
  S.vsh = S.R + bw * (bw + 1) / 2;
  S.prow = S.vsh + kMaxB;
  S.rdiag = S.prow + 2 * kMaxB;
  S.scal = S.rdiag + kMaxB;
  S.vw = S.scal + 8;
  S.red = reinterpret_cast<uint64_t*>(S.vw + NW * 2 * kMaxB);
  S.selpos = reinterpret_cast<int*>(S.red + 2 * NW + 8);
  S.flags = S.selpos + kMaxB;
  S.dest = S.flags + 8;

  const int G = a.G;
  // Interleaved, workgroup w of tile g is block w * ngroups + g: blocks go to
  // the XCDs in turn, so when ngroups is a multiple of 8 a tile's workgroups
  // share one XCD, where a posted word reaches a poller sooner.
  const int g = a.interleave ? (int)blockIdx.x % a.ngroups : (int)blockIdx.x / G;
  const int w = a.interleave ? (int)blockIdx.x / a.ngroups : (int)blockIdx.x - g * G;
  const int tid = threadIdx.x;
  const int l8 = tid & 7;
  const int rg = tid >> 3;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  // the tile (or, for a batch, the problem) of this group
  const double* pA = a.A;
  int64_t plda = a.lda, pk0 = a.k0;
  double* pY = a.Y;
  int64_t pldy = a.ldy;
  prrp_stats* pst = a.stats;
  int32_t* psel = a.sel_out ? a.sel_out + (size_t)g * kMaxB : nullptr;
  int32_t* prounds = a.rounds_out ? a.rounds_out + g : nullptr;
  int tlen, tstart;
  uint64_t* slots;
  if (a.probs != nullptr) {
    const SrrqrProblem& P = a.probs[g];
    pA = P.A; plda = P.lda; pk0 = P.k0;
    pY = P.Y; pldy = P.ldy;
    pst = P.stats;
    psel = P.sel_out;
    prounds = P.rounds_out;
    tlen = P.m;
    tstart = 0;
    slots = P.slots;
  } else {
    tlen = a.tile_len[g];
    tstart = a.tile_start[g];
    slots = a.slots + (size_t)g * a.group_stride;
  }
  const int row0 = w * a.rpw;
  const int nloc = max(0, min(a.rpw, tlen - row0));
  const size_t round_stride = (size_t)G * kPostW;

  // ---- restore the sentinels of the slot set used by the previous launch
  // (a batch: each problem's own previous set, by that problem's workgroups)
  if (a.probs != nullptr) {
    const SrrqrProblem& P = a.probs[g];
    if (P.clear_base != nullptr) {
      const int nthr = G * NT;
      const int gt = w * NT + tid;
      const int per_post = post_width(P.clear_bw);
      const size_t total = (size_t)(*P.clear_rounds) * P.clear_G * per_post;
      for (size_t e = gt; e < total; e += nthr) {
        const size_t post = e / per_post;
        const int wd = (int)(e - post * per_post);
        P.clear_base[post * kPostW + wd] = kKeySent;
      }
    }
  } else if (a.clear_base != nullptr) {
    const int nthr = gridDim.x * NT;
    const int gt = blockIdx.x * NT + tid;
    const int per_post = post_width(a.clear_bw);
    for (int cg = 0; cg < a.clear_ngroups; ++cg) {
      const int used = a.clear_rounds[cg];
      uint64_t* base = a.clear_base + (size_t)cg * a.clear_group_stride;
      const size_t total = (size_t)used * a.clear_G * per_post;
      for (size_t e = gt; e < total; e += nthr) {
        const size_t post = e / per_post;
        const int wd = (int)(e - post * per_post);
        base[post * kPostW + wd] = kKeySent;
      }
    }
  }

  // ---- load this workgroup's rows
  double x[RPT][CPT];
  int tpos[RPT];
  bool live[RPT], chosen[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int lr = rg + kRowGroups * q;
    tpos[q] = row0 + lr;
    live[q] = lr < nloc;
    chosen[q] = false;
    int64_t prow_idx = 0;
    if (live[q]) prow_idx = a.row_list ? a.row_list[tstart + tpos[q]] : tstart + tpos[q];
    const double* src = a.panel ? a.panel + prow_idx * a.ldp : pA + (pk0 + prow_idx) * plda + pk0;
#pragma unroll
    for (int k = 0; k < CPT; ++k) {
      const int c = l8 + 8 * k;
      x[q][k] = (live[q] && c < bw) ? ld_g(src + c) : 0.0;
    }
  }
  if (tid < kMaxB) { S.vsh[tid] = 0.0; }
  if (tid < 8) S.flags[tid] = 0;
  __syncthreads();

  int bad = 0;
  const bool multi = G > 1;
  if (tid < 2 * kMaxB) S.prow[tid] = 0.0;
  __syncthreads();

  // ================================================================ QR steps
  // Step s: (1) every wave rebuilds reflector H_{s-1} from the winner row of
  // step s-1 (in LDS) and applies it to its unselected rows; (2) squared
  // norms of the trailing parts, best candidate of the workgroup (barrier);
  // (3) post it, and every wave polls the G posted keys itself; (4) the
  // winning row is brought into LDS (barrier).
  for (int s = 0; s <= bw; ++s) {
    if (s > 0) {
      const int sp = s - 1;
      const int c0 = sp + lane, c1 = sp + lane + 64;
      const double x0 = S.prow[c0];           // zero past bw
      const double x1 = S.prow[c1];
      const double head = S.prow[sp];
      // formed by the pivot row's owner while its key travelled
      const double alpha = S.scal[4];
      const double beta = S.scal[5];
      const double v0 = head - alpha;
      if (wave == 1) {
        for (int i = lane; i < sp; i += 64) S.R[sp * (sp + 1) / 2 + i] = S.prow[i];
        if (lane == 0) S.R[sp * (sp + 1) / 2 + sp] = alpha;
      }
      // the reflector, zero left of sp, through this wave's own LDS vector
      // (written and read by the same wave: no barrier, no per-element selects)
      double* vw = S.vw + wave * 2 * kMaxB;
      vw[c0] = (c0 == sp) ? v0 : x0;
      vw[c1] = x1;
      if (lane < sp) vw[lane] = 0.0;
      if (lane + 64 < sp) vw[lane + 64] = 0.0;
      double vr[CPT];
#pragma unroll
      for (int k = 0; k < CPT; ++k) vr[k] = vw[l8 + 8 * k];
      // branch-free over the rows (so that their chains interleave); rows
      // already chosen, and rows past the tile, take f = 0 and keep their values
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        double dd[4] = {0.0, 0.0, 0.0, 0.0};     // independent chains
#pragma unroll
        for (int k = 0; k < CPT; ++k) dd[k & 3] = fma(vr[k], x[q][k], dd[k & 3]);
        const double d = sum8((dd[0] + dd[1]) + (dd[2] + dd[3]));
        const double f = (live[q] && !chosen[q]) ? beta * d : 0.0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) x[q][k] = fma(-f, vr[k], x[q][k]);
      }
    }
    if (s == bw) break;

    int p;              // tile position of this step's pivot
    int wbad = 0;
    int cq = -1;        // the workgroup's candidate among this thread's rows
    double c_alpha = 0.0, c_beta = 0.0;   // the reflector it would define
    {
      uint64_t best = 0;
      // 0/1 masks of the trailing columns c >= s, shared by the rows (columns
      // past bw hold zeros); the high word alone encodes 1.0 or 0.0
      double cm[CPT];
#pragma unroll
      for (int k = 0; k < CPT; ++k)
        cm[k] = __hiloint2double((l8 + 8 * k >= s) ? 0x3FF00000 : 0, 0);
      double nuq[RPT];
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        double nn[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          const double xm = x[q][k] * cm[k];
          nn[k & 3] = fma(xm, xm, nn[k & 3]);
        }
        nuq[q] = sum8((nn[0] + nn[1]) + (nn[2] + nn[3]));
        const uint64_t key = (live[q] && !chosen[q]) ? make_key(nuq[q], (uint32_t)tpos[q]) : 0ull;
        best = key > best ? key : best;
      }
      best = wave_max_rows(best);
      if (lane == 0) S.red[wave] = best;
      __syncthreads();
      uint64_t wkey = S.red[0];
#pragma unroll
      for (int i = 1; i < NW; ++i) wkey = umax(wkey, S.red[i]);
      uint64_t gkey = wkey;
      uint64_t* post_r = slots + (size_t)s * round_stride;
      // Post my candidate: the key first (it travels while the rest is
      // written; readers poll every word for itself), then the candidate's 8
      // lanes write the row (all 8 CPT words fit the post's width; words past
      // bw are never read) and the alpha, beta of the reflector it defines:
      // nrm^2 is its trailing norm nu, alpha = -sign(head) nrm and
      // beta = 2 / (v^T v) = 1 / (nrm (nrm + |head|)).
      if (multi && tid == 0) st_dev(post_r + (size_t)w * kPostW, wkey);
#pragma unroll
      for (int q = 0; q < RPT; ++q)
        if (wkey != 0 && live[q] && !chosen[q] && (uint32_t)tpos[q] == key_index(wkey)) cq = q;
      if (cq >= 0) {
        double xv[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          xv[k] = x[0][k];
#pragma unroll
          for (int q = 1; q < RPT; ++q) xv[k] = (cq == q) ? x[q][k] : xv[k];
        }
        uint64_t* dst = post_r + (size_t)w * kPostW + 2 + l8;
        if (multi) {
#pragma unroll
          for (int k = 0; k < CPT; ++k) st_dev(dst + 8 * k, (uint64_t)__double_as_longlong(xv[k]));
        }
        double xs = xv[0];                  // column s sits on lane s & 7
#pragma unroll
        for (int k = 1; k < CPT; ++k) xs = (k == (s >> 3)) ? xv[k] : xs;
        const double head = __shfl(xs, (lane & ~7) | (s & 7), 64);
        double nuv = nuq[0];
#pragma unroll
        for (int q = 1; q < RPT; ++q) nuv = (cq == q) ? nuq[q] : nuv;
        const double nrm = sqrt(nuv);
        c_alpha = (nrm == 0.0) ? 0.0 : -copysign(nrm, head);
        c_beta = (nrm == 0.0) ? 0.0 : 1.0 / (nrm * (nrm + fabs(head)));
        if (multi && l8 == 0) {
          st_dev(dst + 8 * CPT, (uint64_t)__double_as_longlong(c_alpha));
          st_dev(dst + 8 * CPT + 1, (uint64_t)__double_as_longlong(c_beta));
        }
      }
      if (multi) {
        // wave 0 polls the G keys (one poller per workgroup keeps the fabric
        // traffic low) and shares the maximum through LDS
        if (wave == 0) {
          uint64_t kv = 0;
          if (G <= 64) {
            if (lane < G) kv = poll_word(post_r + (size_t)lane * kPostW, a.abort_flag, &wbad);
          } else {
            for (int m0 = 0; m0 < G; m0 += 256)
              kv = umax(kv, poll_keys(post_r + (size_t)m0 * kPostW, kPostW, min(G - m0, 256), lane,
                                      a.abort_flag, &wbad));
          }
          kv = wave_max_key(kv);
          if (lane == 0) { S.red[2 * NW] = kv; S.flags[4] = wbad; }
        }
        __syncthreads();
        gkey = S.red[2 * NW];
        wbad = S.flags[4];
      }
      if (gkey == 0 && !wbad) {      // fewer rows than columns: not a valid tile
        if (tid == 0) set_info(pst, -2);
        wbad = 1;
      }
      if (key_nonfinite(gkey) && tid == 0) set_info(pst, -1);
      if ((gkey >> kDropBits) == 0 && tid == 0) {     // exactly zero residual
        S.flags[1] = 1;
        if (a.report_rank) set_info(pst, (int32_t)(pk0 + s + 1));
      }
      p = (int)key_index(gkey);
    }

    // bring the pivot row into LDS
    int owner = p / a.rpw;
    if (owner >= G || wbad) owner = G;           // only after a failed wait
    uint64_t* post_r = slots + (size_t)s * round_stride;
    if (owner == w) {
#pragma unroll
      for (int q = 0; q < RPT; ++q) {
        if (live[q] && tpos[q] == p) {
#pragma unroll
          for (int k = 0; k < CPT; ++k) {
            const int c = l8 + 8 * k;
            if (c < bw) S.prow[c] = x[q][k];
          }
          chosen[q] = true;
        }
      }
      if (cq >= 0 && l8 == 0) { S.scal[4] = c_alpha; S.scal[5] = c_beta; }
    } else if (owner < G) {
      if (tid < bw) {
        const uint64_t v = poll_word(post_r + (size_t)owner * kPostW + 2 + tid, a.abort_flag, &wbad);
        S.prow[tid] = __longlong_as_double((long long)v);
      }
      if (tid >= NT - 2) {
        const int j = tid - (NT - 2);
        const uint64_t v =
            poll_word(post_r + (size_t)owner * kPostW + 2 + 8 * CPT + j, a.abort_flag, &wbad);
        S.scal[4 + j] = __longlong_as_double((long long)v);
      }
    }
    if (wbad) S.flags[0] = 1;
    if (tid == 0) S.selpos[s] = p;
    __syncthreads();
    if (S.flags[0]) break;
  }
  // the last pass wrote R's last column (wave 1) and no barrier followed it
  __syncthreads();

  // After a failed wait the launch's outputs are not formed; in-range
  // placeholders keep the kernels that read them inside the panel.
  auto abandon = [&]() {
    if (tid == 0) {
      set_info(pst, -2);
      st_dev_u32(a.abort_flag, 1u);
    }
    if (psel && w == 0 && tid < bw && tlen > 0) {
      const int t = min(tid, tlen - 1);
      psel[tid] = a.row_list ? a.row_list[tstart + t] : tstart + t;
    }
    if (a.plan_mv) {
      if (w == 0 && tid == 0) a.plan_mv[4 * kMaxB] = 0;
      for (int t = row0 + tid; t < row0 + nloc; t += NT)
        if (t >= bw) a.srcmap[t - bw] = t;
    }
  };
  if (S.flags[0]) {
    abandon();
    return;
  }

  int rounds_used = bw;
  int swaps = 0;
  const bool rank_def = S.flags[1] != 0;
  double mmax_local = 0.0;

  if (!rank_def && tlen > bw) {
    // ============================================= M = R11^-1 R12 per row
    if (tid < bw) S.rdiag[tid] = 1.0 / S.R[tid * (tid + 1) / 2 + tid];
    __syncthreads();
    // (the column block kk is unrolled so that every index into x is static;
    // the 8 columns of a block stay a loop)
#pragma unroll
    for (int kk = CPT - 1; kk >= 0; --kk) {
#pragma unroll 1
      for (int li = 7; li >= 0; --li) {
        const int i = 8 * kk + li;
        if (i >= bw) continue;
        double rcol[CPT];
        // R(c, i) for c < i; the unguarded reads stay inside the packed array
#pragma unroll
        for (int k = 0; k <= kk; ++k) rcol[k] = S.R[i * (i + 1) / 2 + l8 + 8 * k];
#pragma unroll
        for (int k = 0; k <= kk; ++k) rcol[k] = (l8 + 8 * k < i) ? rcol[k] : 0.0;
        const double di = S.rdiag[i];
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const double yi = __shfl(x[q][kk], (lane & ~7) | li, 64) * di;
          if (l8 == li) x[q][kk] = yi;
#pragma unroll
          for (int k = 0; k <= kk; ++k) x[q][k] = fma(-rcol[k], yi, x[q][k]);
        }
      }
    }
    // x[q] now holds column M(:, row) for unselected rows (garbage for chosen)

    {
      // ========================================== exchange loop (Appendix A)
      if (tid < bw) S.vsh[tid] = 0.0;
      for (int e = 0;; ++e) {
        const int r = bw + e;
        // best (magnitude, slot) per row, then best row
        uint64_t best = 0;
        int best_slot = 0;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          uint64_t sk = 0;
#pragma unroll
          for (int k = 0; k < CPT; ++k) {
            const int c = l8 + 8 * k;
            if (c < bw) {
              const uint64_t kk2 = make_key(fabs(x[q][k]), (uint32_t)c);
              sk = kk2 > sk ? kk2 : sk;
            }
          }
          sk = max8_u64(sk);
          if (live[q] && !chosen[q]) {
            const uint64_t rk = ((sk >> kDropBits) << kDropBits) | (kIdxMask - (uint32_t)tpos[q]);
            if (rk > best) { best = rk; best_slot = (int)key_index(sk); }
          }
        }
        const uint64_t wbest = wave_max_rows(best);
        if (lane == 0) S.red[wave] = wbest;
        __syncthreads();
        uint64_t wkey = S.red[0];
#pragma unroll
        for (int i = 1; i < NW; ++i) wkey = S.red[i] > wkey ? S.red[i] : wkey;
        // the owner of the workgroup's best records its slot and row
        const bool own = (best == wkey && wkey != 0);
        uint64_t* post_r = slots + (size_t)r * round_stride;
        if (own && l8 == 0) S.flags[2] = best_slot;
        __syncthreads();
        const int wslot = S.flags[2];
        uint64_t gkey = wkey;
        int gslot = wslot;
        int gowner = w;
        if (multi) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (wkey != 0 && live[q] && !chosen[q] && (uint32_t)tpos[q] == key_index(wkey)) {
#pragma unroll
              for (int k = 0; k < CPT; ++k) {
                const int c = l8 + 8 * k;
                if (c < bw)
                  st_dev(post_r + (size_t)w * kPostW + 2 + c, (uint64_t)__double_as_longlong(x[q][k]));
              }
              if (l8 == 0) st_dev(post_r + (size_t)w * kPostW + 1, (uint64_t)wslot);
            }
          }
          if (tid == 0) st_dev(post_r + (size_t)w * kPostW, wkey);
          uint64_t kv = 0;
          for (int m = tid; m < G; m += NT)
            kv = umax(kv, poll_word(post_r + (size_t)m * kPostW, a.abort_flag, &bad));
          kv = wave_max_u64(kv);
          if (lane == 0) S.red[NW + wave] = kv;
          if (bad) S.flags[0] = 1;
          __syncthreads();
          if (S.flags[0]) break;
          gkey = S.red[NW];
#pragma unroll
          for (int i = 1; i < NW; ++i) gkey = S.red[NW + i] > gkey ? S.red[NW + i] : gkey;
          gowner = (int)key_index(gkey) / a.rpw;
        }
        rounds_used = r + 1;
        const bool violate = gkey != 0 && (gkey >> kDropBits) > a.tau_bits;
        if (!violate) break;
        if (e >= kMaxExchange) {
          if (tid == 0) set_info(pst, -3);
          break;
        }
        const int pj = (int)key_index(gkey);
        // fetch slot and M column of the incoming row
        if (gowner == w) {
#pragma unroll
          for (int q = 0; q < RPT; ++q) {
            if (live[q] && tpos[q] == pj) {
#pragma unroll
              for (int k = 0; k < CPT; ++k) {
                const int c = l8 + 8 * k;
                if (c < bw) S.prow[c] = x[q][k];
              }
            }
          }
          if (tid == 0) S.flags[3] = wslot;
        } else {
          if (tid < bw) {
            const uint64_t v = poll_word(post_r + (size_t)gowner * kPostW + 2 + tid, a.abort_flag, &bad);
            S.prow[tid] = __longlong_as_double((long long)v);
          }
          if (tid == 64) {
            const uint64_t v = poll_word(post_r + (size_t)gowner * kPostW + 1, a.abort_flag, &bad);
            S.flags[3] = (int)v;
          }
          if (bad) S.flags[0] = 1;
        }
        __syncthreads();
        if (S.flags[0]) break;
        gslot = S.flags[3];
        const int out_pos = S.selpos[gslot];
        const double gamma = S.prow[gslot];
        if (tid < bw) S.vsh[tid] = S.prow[tid] - (tid == gslot ? 1.0 : 0.0);   // u = M(:,j) - e_i
        __syncthreads();
        if (tid == 0) S.selpos[gslot] = pj;
        const double ginv = 1.0 / gamma;
        double ur[CPT];
#pragma unroll
        for (int k = 0; k < CPT; ++k) ur[k] = (l8 + 8 * k < bw) ? S.vsh[l8 + 8 * k] : 0.0;
        const int kk_i = gslot >> 3, li_i = gslot & 7;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          double xi = 0.0;
#pragma unroll
          for (int k = 0; k < CPT; ++k) xi = (k == kk_i) ? x[q][k] : xi;
          const double ri = __shfl(xi, (lane & ~7) | li_i, 64);
          if (!live[q]) continue;
          if (tpos[q] == pj) {
            chosen[q] = true;
          } else if (tpos[q] == out_pos) {
            chosen[q] = false;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
              const int c = l8 + 8 * k;
              x[q][k] = ((c == gslot) ? 1.0 : 0.0) - ur[k] * ginv;
            }
          } else if (!chosen[q]) {
            const double f = ri * ginv;
#pragma unroll
            for (int k = 0; k < CPT; ++k) x[q][k] = fma(-ur[k], f, x[q][k]);
          }
        }
        ++swaps;
        __syncthreads();
      }
      if (S.flags[0]) {
        abandon();
        return;
      }
    }
  }

  // ------------------------------------------- moves of Pi_j (whole panel)
  // Pi_j is the sequence of interchanges of positions s and (position of
  // slot s's row) for s = 0 .. bw-1.  Rows outside the top block move only
  // when selected, so (i) slot s's row sits at Q[s] = sel[s] when step s
  // comes, unless sel[s] < s: then it left position sel[s] at step sel[s]
  // for Q[sel[s]], and so on, and Q[s] is the first position >= s on that
  // chain; (ii) a top-block row u left out moves at step u to Q[u], and on
  // along Q until it leaves the top block.  Both chains only increase, so the
  // rounds below end; an unresolved entry waits for the entries it reads.
  const bool fused = a.plan_mv != nullptr;
  if (fused && w * a.rpw < bw) {             // workgroups holding top-block rows
    if (wave == 0) {
      const int e0 = lane, e1 = lane + 64;
      const int s0 = e0 < bw ? S.selpos[e0] : 0;
      const int s1 = e1 < bw ? S.selpos[e1] : 0;
      if (e0 < bw) S.dest[e0] = -1;
      if (e1 < bw) S.dest[e1] = -1;
      if (e0 < bw && s0 < bw) S.dest[s0] = e0;   // selected: not moved out
      if (e1 < bw && s1 < bw) S.dest[s1] = e1;
      // Q by rounds; an unresolved entry holds -1 - (its chase position)
      int v0 = e0 < bw ? (s0 >= e0 ? s0 : -1 - s0) : 0;
      int v1 = e1 < bw ? (s1 >= e1 ? s1 : -1 - s1) : 0;
      for (int it = 0; it <= bw * bw; ++it) {
        if (!__any(v0 < 0 || v1 < 0)) break;
        const int c0 = v0 < 0 ? -1 - v0 : 0;
        const int c1 = v1 < 0 ? -1 - v1 : 0;
        const int a0 = __shfl(v0, c0 & 63, 64), b0 = __shfl(v1, c0 & 63, 64);
        const int a1 = __shfl(v0, c1 & 63, 64), b1 = __shfl(v1, c1 & 63, 64);
        const int q0 = c0 < 64 ? a0 : b0, q1 = c1 < 64 ? a1 : b1;
        if (v0 < 0 && q0 >= 0) v0 = (q0 >= e0) ? q0 : -1 - q0;
        if (v1 < 0 && q1 >= 0) v1 = (q1 >= e1) ? q1 : -1 - q1;
      }
      const bool d0 = e0 < bw && S.dest[e0] == -1;
      const bool d1 = e1 < bw && S.dest[e1] == -1;
      int p0 = e0, p1 = e1;
      for (int it = 0; it <= bw; ++it) {
        const bool m0 = d0 && p0 < bw, m1 = d1 && p1 < bw;
        if (!__any(m0 || m1)) break;
        const int a0 = __shfl(v0, p0 & 63, 64), b0 = __shfl(v1, p0 & 63, 64);
        const int a1 = __shfl(v0, p1 & 63, 64), b1 = __shfl(v1, p1 & 63, 64);
        if (m0) p0 = p0 < 64 ? a0 : b0;
        if (m1) p1 = p1 < 64 ? a1 : b1;
      }
      if (d0) S.dest[e0] = p0;
      if (d1) S.dest[e1] = p1;
      if (w == 0) {
        // top positions take the selected rows in slot order, then the rows
        // left out, in row order
        int32_t* mv = a.plan_mv;
        if (e0 < bw) { mv[e0] = e0; mv[2 * kMaxB + e0] = s0; }
        if (e1 < bw) { mv[e1] = e1; mv[2 * kMaxB + e1] = s1; }
        const uint64_t m0 = __ballot(d0), m1 = __ballot(d1);
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int n0 = __popcll(m0);
        if (d0) {
          const int k = bw + __popcll(m0 & below);
          mv[k] = p0; mv[2 * kMaxB + k] = e0;
        }
        if (d1) {
          const int k = bw + n0 + __popcll(m1 & below);
          mv[k] = p1; mv[2 * kMaxB + k] = e1;
        }
        if (lane == 0) mv[4 * kMaxB] = bw + n0 + __popcll(m1);
      }
    }
    __syncthreads();
  }

  // ----------------------------------------------- outputs: Y rows, max|M|
  // (at the rows' positions after Pi_j when the moves were formed here)
  if (!rank_def && tlen > bw) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (live[q] && !chosen[q]) {
        const int t = (fused && tpos[q] < bw) ? S.dest[tpos[q]] : tpos[q];
        const int64_t pr = a.row_list ? a.row_list[tstart + tpos[q]] : tstart + t;
        const bool in = t >= 0 && t < tlen;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
          const int c = l8 + 8 * k;
          if (c < bw && in) {
            mmax_local = fmax(mmax_local, fabs(x[q][k]));
            if (pY) st_g(pY + pr * pldy + c, x[q][k]);
          }
        }
      }
    }
  }

  if (rank_def && pY) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (live[q] && !chosen[q]) {
        const int t = (fused && tpos[q] < bw) ? S.dest[tpos[q]] : tpos[q];
        const int64_t pr = a.row_list ? a.row_list[tstart + tpos[q]] : tstart + t;
#pragma unroll
        for (int k = 0; k < CPT; ++k)
          if (l8 + 8 * k < bw && t >= 0 && t < tlen) pY[pr * pldy + l8 + 8 * k] = 0.0;
      }
    }
  }
  if (fused && tlen > bw) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      if (live[q] && !chosen[q] && l8 == 0) {
        const int t = tpos[q] < bw ? S.dest[tpos[q]] : tpos[q];
        if (t >= bw && t < tlen) a.srcmap[t - bw] = tpos[q];
      }
    }
  }

  // ------------------------------------------------------ selection, stats
  if (w == 0 && tid < bw) {
    const int sp = S.selpos[tid];
    psel[tid] = a.row_list ? a.row_list[tstart + sp] : tstart + sp;
  }
  if (pst) {
    double m = mmax_local;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0 && m > 0.0 && a.record_block_L) atomic_max_pos(&pst->max_block_L, m);
    if (w == 0 && tid == 0 && swaps > 0)
      __hip_atomic_fetch_add(&pst->swaps, (int64_t)swaps, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (w == 0 && tid == 0) *prounds = rounds_used;
}

// ------------------------------------------------------------- dispatch
// Columns per lane (bw rounded up to 8, 16, 32, 64, 128 columns), the
// workgroup size (1024 threads once a workgroup holds more than 128 rows)
// and rows per thread.
struct Shape { int cpt, nt, rpt; };
// A workgroup of at most 64 rows in a tile of at most 16 workgroups runs
// with 512 threads (one row per thread, two waves per SIMD; measured faster
// on CALU_PRRP's tree nodes), any other of at most 128 rows with 256 (faster
// for a panel spread over 64 workgroups, where the exchange dominates);
// PRRP_SRRQR_THREADS=256 or 512 fixes the size for those.
int mid_threads() {
  static int nt = -1;
  if (nt < 0) {
    const char* e = getenv("PRRP_SRRQR_THREADS");
    const int v = e ? atoi(e) : 0;
    nt = (v == kThreads || v == kThreadsMid) ? v : 0;
  }
  return nt;
}
Shape srrqr_shape(int bw, int rpw, int G) {
  int cpt = (bw + 7) / 8;
  cpt = cpt <= 2 ? (cpt <= 1 ? 1 : 2) : (cpt <= 4 ? 4 : (cpt <= 8 ? 8 : 16));
  int nt = mid_threads();
  if (nt == 0) nt = (rpw <= kThreadsMid / 8 && G <= 16) ? kThreadsMid : kThreads;
  if (rpw > (kThreads / 8) * 4) nt = kThreadsWide;
  return {cpt, nt, (rpw + nt / 8 - 1) / (nt / 8)};
}

#define PRRP_SRRQR_SHAPES(X)                                                                  \
  X(1, 1, kThreads) X(1, 2, kThreads) X(1, 3, kThreads) X(1, 4, kThreads)                   \
  X(2, 1, kThreads) X(2, 2, kThreads) X(2, 3, kThreads) X(2, 4, kThreads)                   \
  X(4, 1, kThreads) X(4, 2, kThreads) X(4, 3, kThreads) X(4, 4, kThreads)                   \
  X(8, 1, kThreads) X(8, 2, kThreads) X(8, 3, kThreads) X(8, 4, kThreads)                   \
  X(16, 1, kThreads) X(16, 2, kThreads) X(16, 3, kThreads) X(16, 4, kThreads)               \
  X(1, 1, kThreadsMid) X(1, 2, kThreadsMid) X(2, 1, kThreadsMid) X(2, 2, kThreadsMid)       \
  X(4, 1, kThreadsMid) X(4, 2, kThreadsMid) X(8, 1, kThreadsMid) X(8, 2, kThreadsMid)       \
  X(16, 1, kThreadsMid) X(16, 2, kThreadsMid)                                               \
  X(1, 2, kThreadsWide) X(2, 2, kThreadsWide) X(4, 2, kThreadsWide) X(8, 2, kThreadsWide)

#define PRRP_SRRQR_CASE(C, R, T)                                                           \
  if (sh.cpt == C && sh.rpt == R && sh.nt == T) {                                          \
    hipLaunchKernelGGL((srrqr_kernel<C, R, T>), dim3(a.ngroups * a.G), dim3(T), smem,     \
                       stream, a);                                                         \
    return hipGetLastError();                                                              \
  }

hipError_t launch_srrqr(const SrrqrArgs& a, hipStream_t stream) {
  const Shape sh = srrqr_shape(a.bw, a.rpw, a.G);
  const size_t smem = srrqr_smem_bytes(a.bw, sh.nt);
  PRRP_SRRQR_SHAPES(PRRP_SRRQR_CASE)
  return hipErrorInvalidValue;
}

int srrqr_max_rpw() { return kRowsWide; }

#define PRRP_SRRQR_OCC(C, R, T)                                                               \
  if (sh.cpt == C && sh.rpt == R && sh.nt == T)                                               \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, srrqr_kernel<C, R, T>, T, smem);

// Workgroups of one instance that a compute unit holds at once.
hipError_t srrqr_blocks_per_cu(int bw, int rpw, int G, int* blocks) {
  const Shape sh = srrqr_shape(bw, rpw, G);
  const size_t smem = srrqr_smem_bytes(bw, sh.nt);
  PRRP_SRRQR_SHAPES(PRRP_SRRQR_OCC)
  return hipErrorInvalidValue;
}

#define PRRP_SRRQR_ATTR(C, R, T)                                                            \
  e = hipFuncSetAttribute((const void*)srrqr_kernel<C, R, T>,                               \
                          hipFuncAttributeMaxDynamicSharedMemorySize,                       \
                          (int)srrqr_smem_bytes(kMaxB, T));                                 \
  if (e != hipSuccess) return e;

hipError_t srrqr_prepare() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e;
  PRRP_SRRQR_SHAPES(PRRP_SRRQR_ATTR)
  done = true;
  return hipSuccess;
}

}  // namespace prrp
