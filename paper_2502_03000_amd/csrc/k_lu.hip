// LU factorisation with partial pivoting and the triangular solves behind
// solve(A, B) and the inv(A)*B rewrite (the xGESV mapping of Sec. I / Sec. II;
// expression (9) of Sec. III).
//
// Right-looking blocked algorithm, panel width 64:
//   panel    one launch factors the n-k x jb panel. Each thread holds one
//            panel row in registers; per column every workgroup publishes
//            its best pivot candidate (largest |a|, lowest position on ties)
//            with the candidate's row as tagged words, reads every
//            workgroup's header, picks the same winner as all the others and
//            reads the winner's row. No grid barrier: the tags make each
//            word self-validating. The participants share one XCD when
//            there are at most 32.
//   laswp    the panel's row interchanges, as a gather of the moved rows, on
//            every column outside the panel and on the row-origin vector.
//   trsm     U12 = L11^-1 A12 as an in-place product with the explicit
//            inverse of the 64 x 64 unit lower block (MFMA GEMM).
//   update   A22 -= L21 U12, a rank-64 update: one MFMA kernel that keeps
//            the whole K range of its A and B tiles in LDS and its C tile in
//            the accumulators (split-BF16 / FP16 updates use the GEMM).
// The solves apply the inverses of the diagonal blocks (kept in the
// workspace): each direction is one launch in which workgroups take (64-row
// block, 16-column chunk) tasks in order, multiply with MFMA and exchange
// solved blocks as tagged words.
// Every wait for another wave's words spins a bounded number of times; a
// timeout sets a status bit instead of hanging, and every wave still reaches
// the end of the kernel.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ew_device.h"
#include "gemm_device.h"
#include "kernels.h"
#include "wave_device.h"

namespace hexla {
namespace k {

namespace {

constexpr int kNB = 64;         // panel width
constexpr int kPT = 256;        // panel threads per workgroup (one row each)
constexpr int kWaves = kPT / 64;  // waves per panel workgroup
constexpr int kMaxG = 64;         // panel workgroups (rows up to kMaxG * kPT)
constexpr int kHdrW = 2;          // header words of a participant's slot
constexpr int kSlotW = kHdrW + 2 * kNB;  // words per slot (FP64 rows: two per value)
constexpr unsigned kNoPos = 0xffff;      // position field of "no candidate"
constexpr unsigned kSpinLimit = 1u << 20;
constexpr int kStatusSingular = 5;  // HEXLA_E_SINGULAR

constexpr int kChainW = 16;                 // FP32 solve: columns per task
constexpr int kChainWords = kNB * kChainW;  // exchange words per solved task
constexpr int kChainCols = 1024;            // columns per pair of solve launches
constexpr unsigned kChainGrid = 512;        // solve workgroups at most (resident)


struct LuWork {
  void* inv;           // [n_panels][2][kNB][kNB]: L11^-1 and U11^-1 of each diagonal block
  uint64_t* slots;     // [2][G][kSlotW] tagged words, by column parity
  int32_t* swap_cnt;   // [n_panels]
  int32_t* swap_list;  // [n_panels][2 * kNB][2]   (dst, src)
  unsigned* tickets;   // [2] task tickets of the forward and backward solves
  uint64_t* xw;        // [chunk][block] solved tasks of the solve, tagged words
};

int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }
size_t slot_bytes(int64_t gmax) { return size_t(2 * gmax * kSlotW) * sizeof(uint64_t); }

LuWork carve(void* work, int64_t n) {
  const int64_t np = cdiv(n, kNB);
  const int64_t gmax = cdiv(n, kPT);
  char* p = static_cast<char*>(work);
  LuWork w;
  w.inv = p;
  p += size_t(np) * 2 * kNB * kNB * sizeof(double);
  w.slots = reinterpret_cast<uint64_t*>(p);
  p += slot_bytes(gmax);
  w.swap_cnt = reinterpret_cast<int32_t*>(p);
  p += size_t(np) * sizeof(int32_t);
  w.swap_list = reinterpret_cast<int32_t*>(p);
  p += size_t(np) * 4 * kNB * sizeof(int32_t);
  // the solve's words are 64-bit atomics: 256-byte aligned (the lists above
  // end on a 4-byte boundary when the panel count is odd)
  p = static_cast<char*>(work) + ((size_t(p - static_cast<char*>(work)) + 255) & ~size_t(255));
  w.tickets = reinterpret_cast<unsigned*>(p);
  p += 256;
  w.xw = reinterpret_cast<uint64_t*>(p);
  return w;
}
// values in the exchange of one pair of launches of the blocked solve (one
// 64-bit word per FP32 value, two per FP64 value)
size_t solve_words(int64_t n, int64_t nrhs) {
  const int64_t chunks = std::min<int64_t>(cdiv(nrhs, kChainW), kChainCols / kChainW);
  return size_t(chunks) * size_t(cdiv(n, kNB)) * kChainWords;
}

// Words other waves read: single-copy atomic 64-bit stores and loads at
// agent scope. Every word carries the (panel, column) tag in its high bits,
// so a reader knows from the word alone whether it holds this column's value.
__device__ __forceinline__ void st_word(uint64_t* p, uint64_t w) {
  __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ld_word(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}
// Bounded wait: false (and the abort flag raised) after kSpinLimit polls or
// when another wave has raised it.
__device__ __forceinline__ bool keep_waiting(unsigned& spins, int32_t* abort_flag) {
  if (++spins > kSpinLimit ||
      __hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
    __hip_atomic_store(abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return false;
  }
  __builtin_amdgcn_s_sleep(1);
  return true;
}

// Panel factorisation. Participants are the workgroups with blockIdx a
// multiple of `stride` (8 places them on one XCD, where the exchange stays
// within one L2); the others return at once. Each thread holds one panel row
// in registers and never hands it to another thread: pos tracks the row's
// current position, and the interchange of positions j and p at step j only
// relabels two rows (GEPP's order, kept as positions). A row is kept rotated
// so that the current column is always v[0]: after step j every row turns
// left by one, and a row still below the pivot appends its multiplier l_j
// where column j left, while a finished row appends column j itself; all
// register indices are static. After jb steps v[c] belongs to column
// (c + jb) mod kNB.
// Per column: the waves' best candidates meet in LDS; the wave holding the
// workgroup's best publishes, as tagged words in the workgroup's slot, the
// candidate's row (its multiplier part zeroed) and the header (|a| key,
// position); wave 0 waits until every participant's header carries this
// column's tag, picks the winner (largest |a|, lowest position), reads the
// winner's row (waiting on its tags too) and shares it through LDS. Slots
// alternate with the column's parity: a workgroup overwrites the parity of
// column j only after every participant has published column j - 1, which
// each does after reading column j - 2. At the end every row is written at
// its final position and the moved rows are listed for laswp.
// T is the storage type, C the type the panel is factored in: a float
// matrix may be factored with FP64 panels (pivots chosen on FP64 values,
// the eliminated panel rounded to float when it is stored).
template <typename T, typename C = T>
__global__ __launch_bounds__(kPT) void panel_kernel(T* __restrict__ A, int64_t lda, int64_t n,
                                                    int64_t k, int jb, int G, int stride,
                                                    uint64_t* slots, unsigned tag0,
                                                    int32_t* swap_cnt, int32_t* swap_list,
                                                    int32_t* status) {
  if (blockIdx.x % stride) return;  // not a participant
  // the panel is the critical path and shares CUs with the trailing update
  // of the previous panel: its waves go first at instruction issue
  __builtin_amdgcn_s_setprio(3);
  constexpr bool kF64 = sizeof(C) == 8;
  __shared__ unsigned s_kh[kWaves], s_kl[kWaves];
  __shared__ int s_kp[kWaves];
  __shared__ C s_row[kNB];  // the candidate row, staged by its owner for its wave
  __shared__ C s_piv[2][kNB];  // the pivot row, by column parity
  __shared__ int s_wp, s_ok;
  const int g = blockIdx.x / stride;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int mp = int(n - k);
  const int r = g * kPT + tid;  // panel row of this thread
  const bool own = r < mp;
  // a wait timed out in an earlier panel: the factorisation is void, exit
  if (__hip_atomic_load(status + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
  C v[kNB];
#pragma unroll
  for (int c = 0; c < kNB; ++c) v[c] = (own && c < jb) ? C(A[(k + r) + (k + c) * lda]) : C(0);
  int pos = own ? r : int(kNoPos);
  if (tid == 0) s_ok = 1;

  // Column j's elimination is split: right after column j's pivot row is
  // known, each row computes only its value in column j + 1, from which the
  // workgroup's candidate for column j + 1 is found and its header published;
  // the rest of the row is eliminated while the other participants' headers
  // travel, and the candidate's row is published after that (readers check
  // every row word's tag, so the row may follow its header).
  C cur = v[0];     // the row's value in the current column
  C l = C(0), last = C(0);
  int wp = 0;
#pragma unroll 1
  for (int j = 0; j < jb; ++j) {
    const uint64_t tag = tag0 + unsigned(j);  // < 2^16
    uint64_t* base = slots + size_t(j & 1) * size_t(G) * kSlotW;
    // 1. the workgroup's candidate: largest key, lowest position
    unsigned kh, kl;
    abs_key(cur, kh, kl);
    const bool cand = own & (pos >= j);
    kh = cand ? kh : 0u;
    kl = cand ? kl : 0u;
    {
      const unsigned mh = wave_max_u32(kh);
      const unsigned ml = kF64 ? wave_max_u32(kh == mh ? kl : 0u) : 0u;
      const int bp = wave_min_i32(((kh == mh) & (kl == ml) & cand) ? pos : 0x7fffffff);
      if (lane == 0) {
        s_kh[wave] = mh;
        s_kl[wave] = ml;
        s_kp[wave] = bp;
      }
    }
    __syncthreads();
    unsigned bh = s_kh[0], bl = s_kl[0];
    int bp = s_kp[0];
#pragma unroll
    for (int q = 1; q < kWaves; ++q) {
      const unsigned h = s_kh[q], ll = s_kl[q];
      const int pp = s_kp[q];
      const bool take = (h > bh) | ((h == bh) & ((ll > bl) | ((ll == bl) & (pp < bp))));
      bh = take ? h : bh;
      bl = take ? ll : bl;
      bp = take ? pp : bp;
    }
    // 2. the header: by lane 0 of the wave holding the candidate (wave 0
    // when the workgroup has none)
    uint64_t* slot = base + size_t(g) * kSlotW;
    const bool holder = __any(pos == bp);
    if (holder && lane == 0) {
      st_word(slot, (tag << 32) | bh);
      st_word(slot + 1, (tag << 48) | (uint64_t(unsigned(bp)) << 32) | bl);
    } else if (bp == 0x7fffffff && wave == 0 && lane == 0) {
      st_word(slot, tag << 32);
      st_word(slot + 1, (tag << 48) | (uint64_t(kNoPos) << 32));
    }
    // 3. the rest of the previous column's elimination: rotate left by one,
    // appending the multiplier (rows below the pivot) or the column itself
    if (j > 0) {
      const C* prow = s_piv[(j - 1) & 1];
      v[0] = cur;
#pragma unroll
      for (int c = 1; c < kNB - 1; ++c) v[c] = v[c + 1] - l * prow[c + 1];
      v[kNB - 1] = last;
    }
    // 4. the candidate's row (its multiplier part zeroed), one value per lane
    if (holder) {
      if (pos == bp) {
#pragma unroll
        for (int c = 0; c < kNB; ++c) s_row[c] = v[c];
      }
      wave_fence();
      const C x = lane < kNB - j ? s_row[lane] : C(0);
      if constexpr (kF64) {
        const uint64_t b = uint64_t(__double_as_longlong(double(x)));
        st_word(slot + kHdrW + 2 * lane, (tag << 32) | (b & 0xffffffffu));
        st_word(slot + kHdrW + 2 * lane + 1, (tag << 32) | (b >> 32));
      } else {
        st_word(slot + kHdrW + lane, (tag << 32) | __float_as_uint(float(x)));
      }
    }
    // 5. wave 0: every participant's header, the winner, the winner's row
    if (wave == 0) {
      unsigned hh = 0u, hl = 0u;
      int hp = 0x7fffffff;
      unsigned spins = 0;
      bool ok = true;
      for (;;) {
        bool got = true;
        if (lane < G) {
          const uint64_t* sq = base + size_t(lane) * kSlotW;
          const uint64_t w0 = ld_word(sq), w1 = ld_word(sq + 1);
          got = ((w0 >> 32) == tag) & ((w1 >> 48) == tag);
          hh = unsigned(w0);
          hl = unsigned(w1);
          const unsigned pp = unsigned(w1 >> 32) & 0xffffu;
          hp = pp == kNoPos ? 0x7fffffff : int(pp);
        }
        if (__all(got)) break;
        if (!keep_waiting(spins, status + 1)) {
          ok = false;
          break;
        }
      }
      int wq = 0x7fffffff, wpp = 0x7fffffff;
      if (ok) {
        const unsigned wh = wave_max_u32(hh);
        const unsigned wl = kF64 ? wave_max_u32(hh == wh ? hl : 0u) : 0u;
        wpp = wave_min_i32(((hh == wh) & (hl == wl)) ? hp : 0x7fffffff);
        wq = wave_min_i32(((hh == wh) & (hl == wl) & (hp == wpp)) ? lane : 0x7fffffff);
        // |pivot| > 0 is a key above (1, 0); otherwise the column is singular
        if (g == 0 && lane == 0 && !((wh > 1u) | ((wh == 1u) & (wl > 0u)))) {
          if (atomicCAS(status, 0, kStatusSingular) == 0) status[2] = int(k + j);
        }
        if (wq >= G) {  // no participant had a candidate: cannot happen while j < n - k
          __hip_atomic_store(status + 1, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          ok = false;
        }
      }
      if (ok) {
        const uint64_t* sw = base + size_t(wq) * kSlotW + kHdrW;
        C pr = C(0);
        spins = 0;
        for (;;) {
          bool got;
          if constexpr (kF64) {
            const uint64_t w0 = ld_word(sw + 2 * lane), w1 = ld_word(sw + 2 * lane + 1);
            got = ((w0 >> 32) == tag) & ((w1 >> 32) == tag);
            pr = C(__longlong_as_double(
                (long long)(((w1 & 0xffffffffu) << 32) | (w0 & 0xffffffffu))));
          } else {
            const uint64_t w0 = ld_word(sw + lane);
            got = (w0 >> 32) == tag;
            pr = C(__uint_as_float(unsigned(w0)));
          }
          if (__all(got)) break;
          if (!keep_waiting(spins, status + 1)) {
            ok = false;
            break;
          }
        }
        s_piv[j & 1][lane] = pr;
      }
      if (lane == 0) {
        s_wp = wpp;
        if (!ok) s_ok = 0;
      }
    }
    __syncthreads();
    if (!s_ok) break;  // the same for every thread of the workgroup
    wp = s_wp;
    const C pivot = s_piv[j & 1][0];
    // 6. interchange positions j and wp; the multiplier and the row's value
    // in column j + 1 (the rest of the elimination follows the next header)
    pos = pos == wp ? j : (pos == j ? wp : pos);
    const bool active = own & (pos > j) & (pivot != C(0));
    l = active ? v[0] / pivot : C(0);
    last = active ? l : v[0];
    cur = v[1] - l * s_piv[j & 1][1];
  }
  if (s_ok) {  // the last column's elimination
    const C* prow = s_piv[(jb - 1) & 1];
    v[0] = cur;
#pragma unroll
    for (int c = 1; c < kNB - 1; ++c) v[c] = v[c + 1] - l * prow[c + 1];
    v[kNB - 1] = last;
  }

  if (!s_ok) return;  // a wait timed out: status[1] is set, the panel is void
  if (own) {
#pragma unroll
    for (int c = 0; c < kNB; ++c) {
      const int col = (c + jb) % kNB;  // every row is rotated by jb
      if (col < jb) A[(k + pos) + (k + col) * lda] = T(v[c]);
    }
    if (pos != r) {
      const int e = atomicAdd(swap_cnt, 1);
      if (e < 2 * kNB) {
        swap_list[2 * e] = int(k + pos);
        swap_list[2 * e + 1] = int(k + r);
      }
    }
  }
}

// Makes x a register value at this point (every load feeding it completed).
template <typename T>
__device__ __forceinline__ void lk_materialize(T& x) {
  asm volatile("" : "+v"(x));
}

// Gather of the moved rows on the columns [lo1, hi1) and [lo2, hi2), and on
// the row-origin vector when `with_rowid`. One wave per column.
template <typename T>
__global__ __launch_bounds__(256) void laswp_kernel(T* __restrict__ A, int64_t lda, int64_t lo1,
                                                    int64_t hi1, int64_t lo2, int64_t hi2,
                                                    int with_rowid, const int32_t* swap_cnt,
                                                    const int32_t* swap_list, int32_t* rowid) {
  const int lane = threadIdx.x & 63;
  const int64_t v = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  const int64_t n1 = hi1 - lo1, n2 = hi2 - lo2;
  if (v >= n1 + n2 + with_rowid) return;
  const int cnt = min(*swap_cnt, 2 * kNB);
  if (v == n1 + n2) {
    int32_t a0 = 0, a1 = 0;
    if (lane < cnt) a0 = rowid[swap_list[2 * lane + 1]];
    if (lane + 64 < cnt) a1 = rowid[swap_list[2 * (lane + 64) + 1]];
    __builtin_amdgcn_wave_barrier();
    if (lane < cnt) rowid[swap_list[2 * lane]] = a0;
    if (lane + 64 < cnt) rowid[swap_list[2 * (lane + 64)]] = a1;
    return;
  }
  T* col = A + (v < n1 ? lo1 + v : lo2 + (v - n1)) * lda;
  T a0 = 0, a1 = 0;
  if (lane < cnt) a0 = col[swap_list[2 * lane + 1]];
  if (lane + 64 < cnt) a1 = col[swap_list[2 * (lane + 64) + 1]];
  __builtin_amdgcn_wave_barrier();
  if (lane < cnt) col[swap_list[2 * lane]] = a0;
  if (lane + 64 < cnt) col[swap_list[2 * (lane + 64)]] = a1;
}

// The critical-path work between two panels in one workgroup, after the
// interchanges on the next nn (<= kNB) columns: R = L11^-1 [I | A12] with
// A12 the nn columns, i.e. L11^-1 (into inv) and U12 (in place). Blocked
// forward substitution over four 16-row blocks with MFMA: D_b = L_bb^-1 by
// substitution (wave 0, lane (b, c) takes column c of D_b), M_bj = D_b L_bj
// for j < b (MFMA), then R_b = D_b B_b - sum_j M_bj R_j. Wave w owns columns
// 32w.. of R (waves 0-1 the identity's, 2-3 those of A12) and keeps them in
// LDS by columns; blocks of one wave depend only on that wave's earlier
// blocks. Loads and stores are coalesced by tile columns.
template <typename T>
__global__ __launch_bounds__(256) void panel_step_kernel(T* __restrict__ A, int64_t lda, int64_t n,
                                                         int64_t k, int jb, int nn,
                                                         T* __restrict__ inv) {
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc_t;
  constexpr int LL = kNB + 16;  // Lc column stride (operand reads without bank conflicts)
  constexpr int LR = kNB + 4;
  __shared__ T Lc[kNB][LL];        // Lc[l][i] = L11(i, l): unit diagonal, identity padding
  __shared__ T Ds[4][16][16 + 4];  // Ds[b][t][i] = D_b(i, t)
  __shared__ T Ms[6][16][16 + 4];  // Ms[p][t][i] = M_bj(i, t), p = b(b-1)/2 + j
  __shared__ T Rs[4][32][LR];      // Rs[w][c][i] = column 32w + c of [I | A12], then of R
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  const int64_t c0 = k + jb;  // first of the nn columns (nn > 0 only when jb == kNB)
  constexpr int PER = kNB * kNB / 256;
  T lv[PER], bv[PER];
#pragma unroll
  for (int q = 0; q < PER; ++q) {  // element (i, l) from thread e % 64
    const int e = tid + 256 * q, i = e % kNB, l = e / kNB;
    lv[q] = A[(k + min(i, jb - 1)) + (k + min(l, jb - 1)) * lda];
    bv[q] = nn > 0 ? A[(k + i) + (c0 + min(l, nn - 1)) * lda] : T(0);
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e % kNB, l = e / kNB;
    Lc[l][i] = (i < jb && l < jb && i > l) ? lv[q] : T(i == l ? 1 : 0);
    Rs[2 + l / 32][l % 32][i] = bv[q];
  }
  __syncthreads();
  if (w == 0) {  // D_b = L_bb^-1, lane (b, c) = (g, l16) builds column c
    T x[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) x[i] = T(i == l16 ? 1 : 0);
#pragma unroll
    for (int l = 0; l < 16; ++l) {
      const T xl = x[l];
#pragma unroll
      for (int i = l + 1; i < 16; ++i) x[i] -= Lc[16 * g + l][16 * g + i] * xl;
    }
#pragma unroll
    for (int i = 0; i < 16; ++i) Ds[g][l16][i] = x[i];
  }
  __syncthreads();
  // M_bj = D_b L_bj: operand A[i][t] = D_b(i, t), B[t][c] = L(16b + t, 16j + c)
  for (int p = w; p < 6; p += 4) {
    const int b = p < 1 ? 1 : p < 3 ? 2 : 3;
    const int j = p - b * (b - 1) / 2;
    acc_t m = acc_t{};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4)
      m = Mf::mma(Ds[b][4 * s4 + g][l16], Lc[16 * j + l16][16 * b + 4 * s4 + g], m);
#pragma unroll
    for (int r = 0; r < 4; ++r) Ms[p][l16][Mf::row(lane, r)] = m[r];
  }
  __syncthreads();
  // R_b = D_b B_b - sum_{j<b} M_bj R_j on this wave's columns (two fragments)
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    acc_t acc[2] = {acc_t{}, acc_t{}};
#pragma unroll
    for (int s4 = 0; s4 < 4; ++s4) {
      const T a = Ds[b][4 * s4 + g][l16];
      const int row = 16 * b + 4 * s4 + g;
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        const T bb = w < 2 ? T(row == 32 * w + 16 * f + l16 ? 1 : 0) : Rs[w][16 * f + l16][row];
        acc[f] = Mf::mma(a, bb, acc[f]);
      }
    }
#pragma unroll
    for (int j = 0; j < b; ++j) {
      const int p = b * (b - 1) / 2 + j;
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const T a = -Ms[p][4 * s4 + g][l16];
#pragma unroll
        for (int f = 0; f < 2; ++f)
          acc[f] = Mf::mma(a, Rs[w][16 * f + l16][16 * j + 4 * s4 + g], acc[f]);
      }
    }
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int r = 0; r < 4; ++r) Rs[w][16 * f + l16][16 * b + Mf::row(lane, r)] = acc[f][r];
    __builtin_amdgcn_s_waitcnt(0);  // the block is in LDS before the next reads it
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int e = tid + 256 * q, i = e % kNB, c = e / kNB;
    inv[e] = Rs[c / 32][c % 32][i];  // (i, c) at i + kNB c
    if (c < nn) A[(k + i) + (c0 + c) * lda] = Rs[2 + c / 32][c % 32][i];
  }
}

// Inverses of the upper diagonal blocks U11 (jb x jb, padded to kNB x kNB
// with the identity) for the backward solve, one thread per column, the
// block in LDS and the column in registers (backward substitution); block p
// of the grid takes rows/columns p * kNB. (The unit lower blocks' inverses
// come from the panel steps.)
template <typename T>
__global__ __launch_bounds__(kNB) void inv_upper_kernel(const T* __restrict__ A, int64_t lda,
                                                        int64_t n, int64_t first_block,
                                                        T* __restrict__ inv) {
  __shared__ T Ls[kNB][kNB + 1];
  const int64_t p = first_block + blockIdx.x;
  const int64_t k = p * kNB;
  const int jb = int(std::min<int64_t>(kNB, n - k));
  const int c = threadIdx.x;
  {
    // thread c loads row c of every column, all loads in flight at once
    // (clamped addresses, the identity padding chosen afterwards); a loop
    // that stored each load before issuing the next waited once per column
    const T* a = A + (k + min(c, jb - 1)) + k * lda;
    T r[kNB];
#pragma unroll
    for (int j = 0; j < kNB; ++j) r[j] = a[int64_t(min(j, jb - 1)) * lda];
#pragma unroll
    for (int j = 0; j < kNB; ++j) Ls[c][j] = (c < jb && j < jb) ? r[j] : T(c == j ? 1 : 0);
  }
  __syncthreads();
  T x[kNB];
#pragma unroll
  for (int i = kNB - 1; i >= 0; --i) {
    T s = i == c ? T(1) : T(0);
#pragma unroll
    for (int l = i + 1; l < kNB; ++l) s -= Ls[i][l] * x[l];
    x[i] = s / Ls[i][i];
  }
  T* out = inv + size_t(p) * 2 * kNB * kNB + kNB * kNB;
#pragma unroll
  for (int i = 0; i < kNB; ++i) out[i + c * kNB] = x[i];
}

// Blocked triangular solve in one launch: T X = X in place for the unit
// lower (forward, L) or upper (backward, U) factor, 64-row blocks, with the
// inverses of the diagonal blocks. Block i of X is T_ii^-1 (X_i - sum_j T_ij
// X_j) over the blocks j solved before it (j < i forward, j > i backward, in
// solve order). A task is one 64-row block of one 16-column chunk;
// workgroups take tasks in solve order (block-major) from a ticket counter,
// so every task a workgroup waits for belongs to a workgroup that is already
// running (no deadlock, whatever the residency). Wave w of the workgroup owns
// rows 16w..16w+15 of the block: its accumulator is one 16x16 MFMA tile,
// X_i(row 16w + Mf::row(l, r), column l%16) in register r of lane l. Per
// dependency the wave multiplies its 16 rows of T_ij (operand A, loaded
// straight from the factor) by the solved chunk X_j (operand B, read from the
// exchange), 16 MFMA steps of k = 4; the loads of the next dependency are
// issued before the products of this one. The last dependency in solve
// order is kept apart: before any wait each wave forms its rows of M_i =
// T_ii^-1 T_i,last, after the others the inverse is applied (one pass of the
// accumulators through LDS) giving Z_i, and once the last block arrives X_i
// = Z_i - M_i X_last is one product on the critical path. A solved block
// goes to the exchange as 64-bit words whose high half is the tag (tag0 +
// block) and whose low half is the FP32 value, or one 32-bit half of the
// FP64 value (two words per value), stored in the order the readers' lanes
// load them (value 64 s + l: row 4 s + l/16, column l%16), so a reader knows
// from each word alone whether it holds this solve's value: no flag and no
// wait for store completion. The exchange and the tickets start at zero (tags start at 1).
// Padding rows and columns are exact zeros. Every wait is bounded: a timeout
// raises status[1] and the workgroup exits.
// TRANS: the factor is the transpose of the stored lower triangle (L^T of a
// Cholesky factor, backward): T_ij = L_ji^T, read along rows of L, and the
// diagonal blocks' inverses are read transposed. The inverse of block i is
// at inv + i inv_stride (column-major 64 x 64).
template <typename T, bool UPPER, bool TRANS = false>
__global__ __launch_bounds__(256) void chain_solve_kernel(
    const T* __restrict__ LU, int64_t lda, int64_t n, const T* __restrict__ inv,
    int64_t inv_stride, T* __restrict__ X, int64_t ldx, int64_t c_begin, int64_t nrhs, int chunks,
    uint64_t* xw, unsigned* ticket, unsigned tag0, int32_t* status) {
  using Mf = Mfma<T>;
  using acc_t = typename Mf::acc_t;
  constexpr int WPV = sizeof(T) / 4;  // exchange words per value
  constexpr size_t kTaskW = size_t(kChainWords) * WPV;
  __shared__ T sacc[kNB][kChainW + 1];
  __shared__ T sM[4][16][kNB + 1];  // a wave's 16 rows of M_i = T_ii^-1 T_i,last
  __shared__ int s_t, s_bad;
  const int nb = int((n + kNB - 1) / kNB);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int l16 = lane & 15, g = lane >> 4;
  if (tid == 0) s_bad = 0;
  for (;;) {
    if (tid == 0) s_t = int(atomicAdd(ticket, 1u));
    __syncthreads();
    const int t = s_t;
    if (t >= nb * chunks) break;
    const int bt = t / chunks, ch = t % chunks;
    const int bi = UPPER ? nb - 1 - bt : bt;
    const int64_t r0 = int64_t(bi) * kNB;
    const int ib = int(std::min<int64_t>(kNB, n - r0));
    const int64_t c0 = c_begin + int64_t(ch) * kChainW;
    const int rc = int(std::min<int64_t>(kChainW, nrhs - c0));
    const uint64_t* xch = xw + size_t(ch) * size_t(nb) * kTaskW;
    const int arow = 16 * w + l16;  // this lane's operand-A row of the block
    const int arow_c = std::min(arow, ib - 1);
    // accumulator: rows 16w + Mf::row(lane, r), column l16 of X_i
    acc_t acc;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + Mf::row(lane, r);
      const T v = X[(r0 + std::min(row, ib - 1)) + (c0 + std::min(l16, rc - 1)) * ldx];
      acc[r] = (row < ib && l16 < rc) ? v : T(0);
    }
    // T_ii^-1 rows 16w.. as operand A (column-major, padded with the identity)
    const T* iv = inv + size_t(bi) * inv_stride;
    T ia[16];
#pragma unroll
    for (int s4 = 0; s4 < 16; ++s4)
      ia[s4] = TRANS ? iv[(4 * s4 + g) + kNB * arow] : iv[arow + kNB * (4 * s4 + g)];
    // operand A of dependency d: -T(r0 + arow, j0 + 4 s + g), zero outside
    auto load_t = [&](int d, T* ta) {
      const int bj = UPPER ? nb - 1 - d : d;
      const int64_t j0 = int64_t(bj) * kNB;
      const int jbj = int(std::min<int64_t>(kNB, n - j0));
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) {
        const int k = 4 * s4 + g;
        const int64_t kc = j0 + std::min(k, jbj - 1);
        const T v = TRANS ? LU[kc + (r0 + arow_c) * lda] : LU[(r0 + arow_c) + kc * lda];
        ta[s4] = (arow < ib && k < jbj) ? -v : T(0);
      }
    };
    auto load_x = [&](int d, uint64_t (*wd)[WPV]) {
      const int bj = UPPER ? nb - 1 - d : d;
      const uint64_t* src = xch + size_t(bj) * kTaskW + WPV * lane;
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4)
#pragma unroll
        for (int h = 0; h < WPV; ++h) wd[s4][h] = ld_word(src + WPV * 64 * s4 + h);
    };
    // -M_i rows 16w.. as operand A, M_i = T_ii^-1 T_i,last for the last
    // dependency (solve order), formed before any wait: the last step is
    // then X_i = Z_i - M_i X_last, one product on the critical path
    T ma[16];
    if (bt > 0) {
      const int bj = UPPER ? nb - 1 - (bt - 1) : bt - 1;
      const int64_t j0 = int64_t(bj) * kNB;
      const int jbj = int(std::min<int64_t>(kNB, n - j0));
#pragma unroll
      for (int fc = 0; fc < 4; ++fc) {
        acc_t mm = acc_t{};
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4) {
          const int k = 4 * s4 + g, c = 16 * fc + l16;  // T_i,last(k, c)
          const int64_t kr = r0 + std::min(k, ib - 1), cc = j0 + std::min(c, jbj - 1);
          const T v = TRANS ? LU[cc + kr * lda] : LU[kr + cc * lda];
          mm = Mf::mma(ia[s4], (k < ib && c < jbj) ? v : T(0), mm);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) sM[w][Mf::row(lane, r)][16 * fc + l16] = mm[r];
      }
      __builtin_amdgcn_s_waitcnt(0);
      __builtin_amdgcn_wave_barrier();
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) ma[s4] = -sM[w][l16][4 * s4 + g];
    }
    bool ok = true;
    T ta[16];
    uint64_t wd[16][WPV];
    const int nd = bt > 0 ? bt - 1 : 0;  // dependencies before the last
    if (nd > 0) {
      load_t(0, ta);
      load_x(0, wd);
    }
    for (int d = 0; d < nd; ++d) {
      T tn[16];
      uint64_t wn[16][WPV];
      if (d + 1 < nd) {
        load_t(d + 1, tn);
        load_x(d + 1, wn);
      }
      // the words of dependency d: re-read those not yet tagged for it
      const int bj = UPPER ? nb - 1 - d : d;
      const unsigned want = tag0 + unsigned(bj);
      const uint64_t* src = xch + size_t(bj) * kTaskW + WPV * lane;
      unsigned spins = 0;
      for (;;) {
        bool mine = true;
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4)
#pragma unroll
          for (int h = 0; h < WPV; ++h) mine &= unsigned(wd[s4][h] >> 32) == want;
        if (__all(mine)) break;
        if (__any(!keep_waiting(spins, status + 1))) {
          ok = false;
          break;
        }
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4)
#pragma unroll
          for (int h = 0; h < WPV; ++h)
            if (unsigned(wd[s4][h] >> 32) != want) wd[s4][h] = ld_word(src + WPV * 64 * s4 + h);
      }
      if (!ok) break;
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) {
        T xv;
        if constexpr (WPV == 2)
          xv = __longlong_as_double(
              (long long)(((wd[s4][1] & 0xffffffffu) << 32) | (wd[s4][0] & 0xffffffffu)));
        else
          xv = __uint_as_float(unsigned(wd[s4][0]));
        acc = Mf::mma(ta[s4], xv, acc);
      }
#pragma unroll
      for (int s4 = 0; s4 < 16; ++s4) {
        ta[s4] = tn[s4];
#pragma unroll
        for (int h = 0; h < WPV; ++h) wd[s4][h] = wn[s4][h];
      }
    }
    if (!ok) s_bad = 1;  // read only after the barrier below
#pragma unroll
    for (int r = 0; r < 4; ++r) sacc[16 * w + Mf::row(lane, r)][l16] = acc[r];
    __syncthreads();
    if (s_bad) break;
    // Z_i = T_ii^-1 acc: operand B[k][j] = acc(4 s + g, l16)
    acc_t x = acc_t{};
#pragma unroll
    for (int s4 = 0; s4 < 16; ++s4) x = Mf::mma(ia[s4], sacc[4 * s4 + g][l16], x);
    if (bt > 0) {  // X_i = Z_i - M_i X_last
      load_x(bt - 1, wd);
      const int bj = UPPER ? nb - 1 - (bt - 1) : bt - 1;
      const unsigned want = tag0 + unsigned(bj);
      const uint64_t* src = xch + size_t(bj) * kTaskW + WPV * lane;
      unsigned spins = 0;
      for (;;) {
        bool mine = true;
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4)
#pragma unroll
          for (int h = 0; h < WPV; ++h) mine &= unsigned(wd[s4][h] >> 32) == want;
        if (__all(mine)) break;
        if (__any(!keep_waiting(spins, status + 1))) {
          ok = false;
          break;
        }
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4)
#pragma unroll
          for (int h = 0; h < WPV; ++h)
            if (unsigned(wd[s4][h] >> 32) != want) wd[s4][h] = ld_word(src + WPV * 64 * s4 + h);
      }
      if (ok) {
#pragma unroll
        for (int s4 = 0; s4 < 16; ++s4) {
          T xv;
          if constexpr (WPV == 2)
            xv = __longlong_as_double(
                (long long)(((wd[s4][1] & 0xffffffffu) << 32) | (wd[s4][0] & 0xffffffffu)));
          else
            xv = __uint_as_float(unsigned(wd[s4][0]));
          x = Mf::mma(ma[s4], xv, x);
        }
      } else {
        s_bad = 1;  // read after the barrier at the end of the task
      }
    }
    uint64_t* dst = xw + size_t(ch) * size_t(nb) * kTaskW + size_t(bi) * kTaskW;
    const uint64_t tag = uint64_t(tag0 + unsigned(bi)) << 32;
#pragma unroll
    for (int r = 0; r < 4 && ok; ++r) {
      const int row = 16 * w + Mf::row(lane, r);  // value 64 s + l holds row 4 s + l/16
      uint64_t* p = dst + size_t(row * kChainW + l16) * WPV;
      if constexpr (WPV == 2) {
        const uint64_t b = uint64_t(__double_as_longlong(double(x[r])));
        st_word(p, tag | (b & 0xffffffffu));
        st_word(p + 1, tag | (b >> 32));
      } else {
        st_word(p, tag | __float_as_uint(float(x[r])));
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + Mf::row(lane, r);
      if (ok && row < ib && l16 < rc) X[(r0 + row) + (c0 + l16) * ldx] = x[r];
    }
    __syncthreads();  // sacc, s_t and s_bad are reused
    if (s_bad) break;
  }
}

template <typename T>
__global__ void gather_rows_kernel(const T* __restrict__ B, int64_t ldb, const int32_t* rowid,
                                   T* __restrict__ X, int64_t ldx, int64_t n, int64_t nrhs) {
  const int64_t total = n * nrhs;
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e % n, c = e / n;
    X[i + c * ldx] = B[rowid[i] + c * ldb];
  }
}

__global__ void iota_kernel(int32_t* p, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    p[i] = int32_t(i);
}

// C -= A B for K <= kNB (the panel's rank-K update): A m x K (lda), B K x n
// (ldb), C m x n (ldc), column-major. One 256-thread workgroup per BT x BT
// tile of C: the C tile is loaded straight into the accumulators, the whole
// K range of the A and B tiles goes to LDS once, and the MFMAs add
// (-B^T) A^T, i.e. the tile is computed transposed (MFMA rows are C's
// columns). That way the accumulator layout puts 16 consecutive rows of one
// column of C in each 16-lane group, so C is read and written in whole
// 64-byte (FP32) or 128-byte (FP64) runs. The traffic is the C tile twice
// plus the A and B tiles once; with K = 64 the kernel is bound by C.
// BTRANS: B is given as its transpose, an n x K matrix (element (k, j) at
// B[j + k ldb]). LOWER: only the tiles on or below the diagonal of a square
// C (tile column <= tile row), workgroup t taking the t-th such tile.
template <typename T, int BT, bool BTRANS = false, bool LOWER = false>
__global__ __launch_bounds__(256) void rank_update_kernel(int64_t m, int64_t n, int K,
                                                          const T* __restrict__ A, int64_t lda,
                                                          const T* __restrict__ B, int64_t ldb,
                                                          T* __restrict__ C, int64_t ldc,
                                                          int tiles_m) {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  constexpr int LD = BT + 1;  // padded LDS rows
  constexpr int WT = BT / 2;  // a wave's part: WT rows x WT columns
  constexpr int F = WT / 16;  // 16 x 16 blocks per side of a wave's part
  __shared__ T sa[kNB][LD];   // A^T: sa[k][row]
  __shared__ T sb[kNB][LD];   // B: sb[k][col]
  int tm = int(blockIdx.x) % tiles_m, tn = int(blockIdx.x) / tiles_m;
  if (LOWER) {  // t = tm (tm + 1) / 2 + tn, tn <= tm
    const int64_t t = blockIdx.x;
    int64_t I = int64_t((sqrt(8.0 * double(t) + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= t) ++I;
    while (I * (I + 1) / 2 > t) --I;
    tm = int(I);
    tn = int(t - I * (I + 1) / 2);
  }
  const int64_t m0 = int64_t(tm) * BT, n0 = int64_t(tn) * BT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wr = wave & 1, wc = wave >> 1;
  const int l16 = lane & 15, g = lane >> 4;
  // 1. the C tile into the accumulators: block (fc, fr) register r holds
  // column n0 + wc*WT + fc*16 + M::row(lane, r), row m0 + wr*WT + fr*16 + l16
  acc_t acc[F][F];
#pragma unroll
  for (int fc = 0; fc < F; ++fc)
#pragma unroll
    for (int fr = 0; fr < F; ++fr)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + wc * WT + fc * 16 + M::row(lane, r);
        const int64_t row = m0 + wr * WT + fr * 16 + l16;
        acc[fc][fr][r] = (row < m && col < n) ? C[row + col * ldc] : T(0);
      }
  // 2. the A and B tiles, all of K, into LDS (zero past m, n and K): every
  // load in flight at once (clamped addresses, zeros chosen afterwards); a
  // loop that stored each value before the next load waited on each one
  {
    constexpr int PER = BT * kNB / 256;
    T va[PER], vb[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int64_t gr = std::min<int64_t>(m0 + e % BT, m - 1);
      va[q] = A[gr + int64_t(min(e / BT, K - 1)) * lda];
      if (BTRANS) {  // along the columns of C, like A along its rows
        const int64_t gc = std::min<int64_t>(n0 + e % BT, n - 1);
        vb[q] = B[gc + int64_t(min(e / BT, K - 1)) * ldb];
      } else {
        const int64_t gc = std::min<int64_t>(n0 + e / kNB, n - 1);
        vb[q] = B[min(e % kNB, K - 1) + gc * ldb];
      }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q;
      const int row = e % BT, ka = e / BT;
      sa[ka][row] = (ka < K && m0 + row < m) ? va[q] : T(0);
      const int kb = BTRANS ? e / BT : e % kNB, col = BTRANS ? e % BT : e / kNB;
      sb[kb][col] = (kb < K && n0 + col < n) ? vb[q] : T(0);
    }
  }
  __syncthreads();
  // 3. acc += (-B^T) A^T: MFMA operand A[i][k] = -B(k, col i) from lane
  // i + 16k, operand B[k][j] = A(row j, k) from lane j + 16k
#pragma unroll 4
  for (int k0 = 0; k0 < kNB; k0 += 4) {
    T a[F], b[F];
#pragma unroll
    for (int f = 0; f < F; ++f) {
      a[f] = -sb[k0 + g][wc * WT + f * 16 + l16];
      b[f] = sa[k0 + g][wr * WT + f * 16 + l16];
    }
#pragma unroll
    for (int fc = 0; fc < F; ++fc)
#pragma unroll
      for (int fr = 0; fr < F; ++fr) acc[fc][fr] = M::mma(a[fc], b[fr], acc[fc][fr]);
  }
  // 4. back to C
#pragma unroll
  for (int fc = 0; fc < F; ++fc)
#pragma unroll
    for (int fr = 0; fr < F; ++fr)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t col = n0 + wc * WT + fc * 16 + M::row(lane, r);
        const int64_t row = m0 + wr * WT + fr * 16 + l16;
        if (row < m && col < n) C[row + col * ldc] = acc[fc][fr][r];
      }
}

template <typename T>
hipError_t syrk_lower_update(int64_t n, int64_t K, const T* W, int64_t ldw, T* C, int64_t ldc,
                             hipStream_t s) {
  constexpr int BT = 64;
  const int64_t tn = cdiv(n, BT);
  if (K > kNB || tn * (tn + 1) / 2 > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((rank_update_kernel<T, BT, true, true>), dim3(unsigned(tn * (tn + 1) / 2)),
                     dim3(256), 0, s, n, n, int(K), W, ldw, W, ldw, C, ldc, int(tn));
  return hipGetLastError();
}

template <typename T>
hipError_t rank_update_bt(int64_t m, int64_t n, int64_t K, const T* A, int64_t lda, const T* Bt,
                          int64_t ldbt, T* C, int64_t ldc, hipStream_t s) {
  constexpr int BT = 64;
  const int64_t tm = cdiv(m, BT), tn = cdiv(n, BT);
  if (K > kNB || tm * tn > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((rank_update_kernel<T, BT, true, false>), dim3(unsigned(tm * tn)), dim3(256),
                     0, s, m, n, int(K), A, lda, Bt, ldbt, C, ldc, int(tm));
  return hipGetLastError();
}

template <typename T>
hipError_t rank_update(int64_t m, int64_t n, int64_t K, const T* A, int64_t lda, const T* B,
                       int64_t ldb, T* C, int64_t ldc, hipStream_t s) {
  // 64 x 64 tiles in both types: the FP32 128 x 128 tile needed 325
  // registers (one wave per SIMD); at 64 x 64 three waves fit
  constexpr int BT = 64;
  const int64_t tm = cdiv(m, BT), tn = cdiv(n, BT);
  if (K > kNB || tm * tn > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((rank_update_kernel<T, BT>), dim3(unsigned(tm * tn)), dim3(256), 0, s, m, n,
                     int(K), A, lda, B, ldb, C, ldc, int(tm));
  return hipGetLastError();
}

// C (m x ncol) -= A (m x kk) * B (kk x ncol): GEMV for one column; the
// factorization's trailing updates (`trailing`) take the rank-K kernel of
// their precision (plain, or split-BF16 / FP16 terms); the rest (the solves'
// narrow updates) the GEMM.
template <typename T>
hipError_t update(int dtype, int64_t m, int64_t ncol, int64_t kk, const T* A, int64_t lda,
                  const T* B, int64_t ldb, T* C, int64_t ldc, hipStream_t s, int prec = 0,
                  bool trailing = false) {
  if (m <= 0 || ncol <= 0 || kk <= 0) return hipSuccess;
  if (ncol == 1) {
    EwProgram epi{};
    epi.n_instr = 3;
    epi.n_leaf = 1;
    epi.rows = m;
    epi.cols = 1;
    epi.op[0] = EW_EXTRA;
    epi.op[1] = EW_LEAF;
    epi.arg[1] = 0;
    epi.op[2] = EW_ADD;
    epi.leaf[0].ptr = C;
    epi.leaf[0].si = 1;
    epi.leaf[0].sj = ldc;
    return gemv_launch(dtype, 0, m, kk, -1.0, A, lda, B, 1, C, 1, &epi, s);
  }
  if (trailing && prec == GEMM_PLAIN && kk <= kNB)
    return rank_update<T>(m, ncol, kk, A, lda, B, ldb, C, ldc, s);
  if constexpr (sizeof(T) == 4) {
    if (trailing && kk <= kNB)
      return rank_update_split_launch(prec, m, ncol, kk, A, lda, B, ldb, C, ldc, s);
  }
  GemmConfig cfg = gemm_choose(dtype, prec, 0, m, ncol, kk);
  cfg.split = 1;
  return gemm_launch(dtype, prec, 0, 0, 0, m, ncol, kk, -1.0, A, lda, B, ldb, 1.0, C, ldc,
                     nullptr, cfg, s);
}

template <typename T>
hipError_t factor_typed(int dtype, int64_t n, T* A, int64_t lda, int32_t* rowid, void* work,
                        int32_t* status, hipStream_t s, int prec, bool panel_fp64,
                        const Lookahead* side) {
  if (n == 0) return hipSuccess;
  if (n > kLuMaxN) return hipErrorInvalidValue;
  const int64_t np = cdiv(n, kNB);
  LuWork w = carve(work, n);
  // Lookahead from three panels on, on the caller's second stream, outside
  // graph capture (a captured sequence stays on one stream).
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  hipError_t ce = hipStreamIsCapturing(s, &cap);
  if (ce != hipSuccess) return ce;
  const bool lookahead = side && side->s && np >= 3 && cap == hipStreamCaptureStatusNone;
  bool pending = false;  // the side stream holds an update the next interchanges must wait for
  // no slot holds a tag of this factorisation yet (tags restart at 1)
  hipError_t e = fill_i32_launch(reinterpret_cast<int32_t*>(w.slots),
                                 int64_t(slot_bytes(cdiv(n, kPT)) / sizeof(int32_t)), 0, s);
  if (e == hipSuccess) e = fill_i32_launch(w.swap_cnt, np, 0, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(iota_kernel, dim3(unsigned(std::min<int64_t>(cdiv(n, 256), 1024))), dim3(256),
                     0, s, rowid, n);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int64_t p = 0; p < np; ++p) {
    const int64_t k = p * kNB;
    const int jb = int(std::min<int64_t>(kNB, n - k));
    const int G = int(cdiv(n - k, kPT));
    // up to 32 participants share one XCD (every 8th workgroup id)
    const int stride = G <= 32 ? 8 : 1;
    int32_t* list = w.swap_list + p * (4 * kNB);
    if (panel_fp64)
      hipLaunchKernelGGL((panel_kernel<T, double>), dim3(G * stride), dim3(kPT), 0, s, A, lda, n, k,
                         jb, G, stride, w.slots, unsigned(p * kNB + 1), w.swap_cnt + p, list,
                         status);
    else
      hipLaunchKernelGGL((panel_kernel<T, T>), dim3(G * stride), dim3(kPT), 0, s, A, lda, n, k, jb,
                         G, stride, w.slots, unsigned(p * kNB + 1), w.swap_cnt + p, list, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (pending) {  // the interchanges touch the columns the side stream updates
      if ((e = hipStreamWaitEvent(s, side->done, 0)) != hipSuccess) return e;
      pending = false;
    }
    // on s: the interchanges on the next panel's columns, L11^-1 and U12 there
    const int64_t right = n - k - jb;
    const int nn = int(std::min<int64_t>(kNB, right));
    const int64_t far = right - nn;
    T* linv = static_cast<T*>(w.inv) + size_t(p) * 2 * kNB * kNB;
    if (nn > 0) {
      hipLaunchKernelGGL((laswp_kernel<T>), dim3(unsigned(cdiv(nn, 4))), dim3(256), 0, s, A, lda,
                         k + jb, k + jb + nn, int64_t(0), int64_t(0), 0, w.swap_cnt + p, list,
                         rowid);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL((panel_step_kernel<T>), dim3(1), dim3(256), 0, s, A, lda, n, k, jb, nn,
                       linv);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // the rest (interchanges on the other columns and the row origins, U12 and
    // the update beyond the next panel's columns) on the side stream when it
    // can run beside the next panel
    const bool use_side = lookahead && far > 0;
    hipStream_t rs = s;
    if (use_side) {
      if ((e = hipEventRecord(side->ready, s)) != hipSuccess) return e;
      if ((e = hipStreamWaitEvent(side->s, side->ready, 0)) != hipSuccess) return e;
      rs = side->s;
    }
    hipLaunchKernelGGL((laswp_kernel<T>), dim3(unsigned(cdiv(k + far + 1, 4))), dim3(256), 0, rs,
                       A, lda, int64_t(0), k, k + jb + nn, n, 1, w.swap_cnt + p, list, rowid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const T* l21 = A + (k + jb) + k * lda;
    if (far > 0) {
      // U12 = L11^-1 A12 as a product with the explicit inverse, in place:
      // a tile's workgroup (BM >= kNB rows, no split) reads all of its
      // columns of A12 before it writes them, and no other workgroup reads them
      T* a12 = A + k + (k + jb + nn) * lda;
      GemmConfig tc = gemm_choose(dtype, 0, 0, jb, far, jb);
      tc.split = 1;
      e = gemm_launch(dtype, 0, 0, 0, 0, jb, far, jb, 1.0, linv, kNB, a12, lda, 0.0, a12, lda,
                      nullptr, tc, rs);
      if (e != hipSuccess) return e;
      e = update<T>(dtype, right, far, jb, l21, lda, a12, lda, A + (k + jb) + (k + jb + nn) * lda,
                    lda, rs, prec, true);
      if (e != hipSuccess) return e;
    }
    if (use_side) {
      if ((e = hipEventRecord(side->done, side->s)) != hipSuccess) return e;
      pending = true;
    }
    // A22 -= L21 U12 on the next panel's columns, on s and in the storage
    // precision (the next panel waits for it)
    if (nn > 0) {
      e = update<T>(dtype, right, nn, jb, l21, lda, A + k + (k + jb) * lda, lda,
                    A + (k + jb) + (k + jb) * lda, lda, s, GEMM_PLAIN, true);
      if (e != hipSuccess) return e;
    }
  }
  if (pending && (e = hipStreamWaitEvent(s, side->done, 0)) != hipSuccess) return e;
  // every U11^-1, for the solves (each L11^-1 came with its panel step)
  hipLaunchKernelGGL((inv_upper_kernel<T>), dim3(unsigned(np)), dim3(kNB), 0, s, A, lda, n,
                     int64_t(0), static_cast<T*>(w.inv));
  return hipGetLastError();
}

// One direction of the blocked triangular solve over all columns of X, one
// launch per 1024 columns: mode 0 lower (forward), 1 upper (backward), 2
// the transpose of the stored lower triangle (backward). tickets (two
// counters) and xw (the exchange) come from the caller's workspace; tag0
// distinguishes a second direction sharing the same exchange (tags of the
// first: 1..nb, the second: nb+1..2nb); the words are cleared with the
// first direction.
template <typename T>
hipError_t chain_run(int mode, int64_t n, int64_t nrhs, const T* M, int64_t ldm, const T* inv,
                     int64_t inv_stride, T* X, int64_t ldx, unsigned* tickets, uint64_t* xw,
                     bool second, int32_t* status, hipStream_t s) {
  const int64_t nb = cdiv(n, kNB);
  constexpr int64_t wpv = sizeof(T) / 4;
  hipError_t e = hipSuccess;
  for (int64_t cb = 0; cb < nrhs; cb += kChainCols) {
    const int64_t cols = std::min<int64_t>(nrhs - cb, kChainCols);
    const int chunks = int(cdiv(cols, kChainW));
    // resident workgroups: two waves per SIMD in FP32, one in FP64
    const unsigned grid =
        unsigned(std::min<int64_t>(nb * chunks, sizeof(T) == 8 ? kChainGrid / 2 : kChainGrid));
    if (!second || cb > 0) {  // fresh tickets and words
      e = fill_i32_launch(reinterpret_cast<int32_t*>(tickets),
                          256 / 4 + 2 * wpv * int64_t(chunks) * nb * kChainWords, 0, s);
      if (e != hipSuccess) return e;
    }
    unsigned* tk = tickets + (second ? 1 : 0);
    const unsigned tag0 = second ? unsigned(nb + 1) : 1u;
    if (mode == 0)
      hipLaunchKernelGGL((chain_solve_kernel<T, false>), dim3(grid), dim3(256), 0, s, M, ldm, n,
                         inv, inv_stride, X, ldx, cb, nrhs, chunks, xw, tk, tag0, status);
    else if (mode == 1)
      hipLaunchKernelGGL((chain_solve_kernel<T, true>), dim3(grid), dim3(256), 0, s, M, ldm, n,
                         inv, inv_stride, X, ldx, cb, nrhs, chunks, xw, tk, tag0, status);
    else
      hipLaunchKernelGGL((chain_solve_kernel<T, true, true>), dim3(grid), dim3(256), 0, s, M,
                         ldm, n, inv, inv_stride, X, ldx, cb, nrhs, chunks, xw, tk, tag0, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Forward and backward substitution, each one launch of chain_solve_kernel
// per 1024 columns.
template <typename T>
hipError_t solve_typed(int64_t n, int64_t nrhs, const T* LU, int64_t lda, const int32_t* rowid,
                       void* work, const T* B, int64_t ldb, T* X, int64_t ldx, int32_t* status,
                       hipStream_t s) {
  if (n == 0 || nrhs == 0) return hipSuccess;
  hipLaunchKernelGGL((gather_rows_kernel<T>), dim3(unsigned(std::min<int64_t>(cdiv(n * nrhs, 256), 2048))),
                     dim3(256), 0, s, B, ldb, rowid, X, ldx, n, nrhs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  LuWork w = carve(work, n);
  const T* inv = static_cast<const T*>(w.inv);
  for (int64_t cb = 0; cb < nrhs; cb += kChainCols) {
    const int64_t cols = std::min<int64_t>(nrhs - cb, kChainCols);
    T* xc = X + cb * ldx;
    e = chain_run<T>(0, n, cols, LU, lda, inv, 2 * kNB * kNB, xc, ldx, w.tickets, w.xw, false,
                     status, s);
    if (e == hipSuccess)
      e = chain_run<T>(1, n, cols, LU, lda, inv + kNB * kNB, 2 * kNB * kNB, xc, ldx, w.tickets,
                       w.xw, true, status, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

size_t lu_workspace_bytes(int dtype, int64_t n, int64_t nrhs) {
  const int64_t np = cdiv(std::max<int64_t>(n, 1), kNB);
  const int64_t gmax = cdiv(std::max<int64_t>(n, 1), kPT);
  size_t b = size_t(np) * 2 * kNB * kNB * sizeof(double);
  b += slot_bytes(gmax);
  b += size_t(np) * sizeof(int32_t);
  b += size_t(np) * 4 * kNB * sizeof(int32_t);
  b = (b + 255) & ~size_t(255);
  b += 256;  // tickets
  // the solve's exchange (one 64-bit word per FP32 value, two per FP64 value)
  if (nrhs > 0)
    b += solve_words(std::max<int64_t>(n, 1), nrhs) * sizeof(uint64_t) * (dtype == 0 ? 2 : 1);
  return (b + 255) & ~size_t(255);
}

size_t tri_chain_work_bytes(int dtype, int64_t n, int64_t nrhs) {
  if (n <= 0 || nrhs <= 0) return 0;
  return 256 + solve_words(n, nrhs) * sizeof(uint64_t) * (dtype == 0 ? 2 : 1);
}

hipError_t tri_chain_launch(int dtype, int64_t n, int64_t nrhs, const void* M, int64_t ldm,
                            int mode1, const void* inv1, int64_t stride1, int mode2,
                            const void* inv2, int64_t stride2, void* X, int64_t ldx, void* work,
                            int32_t* status, hipStream_t s) {
  if (n <= 0 || nrhs <= 0) return hipSuccess;
  if (n > kLuMaxN || mode1 < 0 || mode1 > 2 || mode2 < -1 || mode2 > 2 ||
      (reinterpret_cast<uintptr_t>(work) & 255))
    return hipErrorInvalidValue;
  unsigned* tickets = static_cast<unsigned*>(work);
  uint64_t* xw = reinterpret_cast<uint64_t*>(static_cast<char*>(work) + 256);
  hipError_t e = hipSuccess;
  // per 1024 columns: the first direction, then the second on the same words
  for (int64_t cb = 0; cb < nrhs && e == hipSuccess; cb += kChainCols) {
    const int64_t cols = std::min<int64_t>(nrhs - cb, kChainCols);
    for (int d = 0; d < 2 && e == hipSuccess; ++d) {
      const int mode = d == 0 ? mode1 : mode2;
      if (mode < 0) break;
      const void* inv = d == 0 ? inv1 : inv2;
      const int64_t stride = d == 0 ? stride1 : stride2;
      if (dtype == 0)
        e = chain_run<double>(mode, n, cols, static_cast<const double*>(M), ldm,
                              static_cast<const double*>(inv), stride,
                              static_cast<double*>(X) + cb * ldx, ldx, tickets, xw, d == 1,
                              status, s);
      else
        e = chain_run<float>(mode, n, cols, static_cast<const float*>(M), ldm,
                             static_cast<const float*>(inv), stride,
                             static_cast<float*>(X) + cb * ldx, ldx, tickets, xw, d == 1, status,
                             s);
    }
  }
  return e;
}

hipError_t rank_update_bt_launch(int dtype, int64_t m, int64_t n, int64_t K, const void* A,
                                 int64_t lda, const void* Bt, int64_t ldbt, void* C, int64_t ldc,
                                 hipStream_t s) {
  if (m <= 0 || n <= 0 || K <= 0) return hipSuccess;
  return dtype == 0 ? rank_update_bt<double>(m, n, K, static_cast<const double*>(A), lda,
                                             static_cast<const double*>(Bt), ldbt,
                                             static_cast<double*>(C), ldc, s)
                    : rank_update_bt<float>(m, n, K, static_cast<const float*>(A), lda,
                                            static_cast<const float*>(Bt), ldbt,
                                            static_cast<float*>(C), ldc, s);
}

hipError_t syrk_lower_update_launch(int dtype, int64_t n, int64_t K, const void* W, int64_t ldw,
                                   void* C, int64_t ldc, hipStream_t s) {
  if (n <= 0 || K <= 0) return hipSuccess;
  return dtype == 0 ? syrk_lower_update<double>(n, K, static_cast<const double*>(W), ldw,
                                                static_cast<double*>(C), ldc, s)
                    : syrk_lower_update<float>(n, K, static_cast<const float*>(W), ldw,
                                               static_cast<float*>(C), ldc, s);
}

hipError_t lu_factor_launch(int dtype, int64_t n, void* A, int64_t lda, int32_t* rowid,
                            void* work, int32_t* status, hipStream_t s, const Lookahead* side,
                            int update_precision, bool panel_fp64) {
  return dtype == 0
             ? factor_typed<double>(0, n, static_cast<double*>(A), lda, rowid, work, status, s, 0,
                                    false, side)
             : factor_typed<float>(1, n, static_cast<float*>(A), lda, rowid, work, status, s,
                                   update_precision, panel_fp64, side);
}

hipError_t lu_solve_launch(int dtype, int64_t n, int64_t nrhs, const void* LU, int64_t lda,
                           const int32_t* rowid, void* work, const void* B, int64_t ldb, void* X,
                           int64_t ldx, int32_t* status, hipStream_t s) {
  return dtype == 0
             ? solve_typed<double>(n, nrhs, static_cast<const double*>(LU), lda, rowid, work,
                                   static_cast<const double*>(B), ldb, static_cast<double*>(X), ldx,
                                   status, s)
             : solve_typed<float>(n, nrhs, static_cast<const float*>(LU), lda, rowid, work,
                                  static_cast<const float*>(B), ldb, static_cast<float*>(X), ldx,
                                  status, s);
}

}  // namespace k
}  // namespace hexla
