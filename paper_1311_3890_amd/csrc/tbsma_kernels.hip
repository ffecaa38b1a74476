// HIP kernels of libtbsma for gfx950 (MI355X): cell binning, Verlet lists,
// the two TB-SMA force passes (FP64 and mixed precision), the BAOAB
// integrator with rigid grips, per-replica reductions and initial state.
//
// One thread per atom slot; a wavefront (64 lanes) is one tile of slots and
// never straddles two replicas, so per-replica sums are exact per wave and
// need no atomics.  Kernels over slots use 256-thread blocks.
#include <algorithm>

#include "tbsma_device.hpp"
#include "tbsma_kernels.hpp"

namespace tbsma {

// ---------------------------------------------------------------------------
// workspace / small helpers
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long *p, int64_t n,
                           unsigned long long v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_set_step(int64_t *step, int64_t v) { *step = v; }

// Quantised copy of the positions (mixed precision): q = rint((x - o) 2^qbits)
// about the centre o of the replica's grid.
__device__ __forceinline__ int quant1(double v, double o, double qs,
                                      bool &out) {
  double t = rint((v - o) * qs);
  if (!(t > -2147483000.0 && t < 2147483000.0)) {
    out = true;
    t = t > 0.0 ? 2147483000.0 : -2147483000.0;
  }
  return (int)t;
}

__device__ __forceinline__ int4 quantise(const Dev &S, int r, int64_t i,
                                         double x, double y, double z,
                                         bool &out) {
  const int32_t *gd = S.grid_dim + 3 * r;
  const double *lo = S.grid_lo + 3 * r;
  double hc = 0.5 * S.cell;
  int4 q;
  q.x = quant1(x, lo[0] + hc * gd[0], S.qscale, out);
  q.y = quant1(y, lo[1] + hc * gd[1], S.qscale, out);
  q.z = quant1(z, lo[2] + hc * gd[2], S.qscale, out);
  q.w = 0;  // g_i of these positions: written by the next density pass
  S.qpos[i] = q;
  return q;
}

__global__ void __launch_bounds__(kBlock) k_quantise(Dev S) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= S.N) return;
  int r = S.tile_rep[i / kTile];
  bool out = false;
  if (S.flag[i] == 3) {
    S.qpos[i] = make_int4(0, 0, 0, 0);
    return;
  }
  quantise(S, r, i, S.x[i], S.y[i], S.z[i], out);
  if (out) atomicOr(&S.wstatus[r], 4u);
}

// ---------------------------------------------------------------------------
// cell binning: count -> per-replica scan -> fill -> per-cell sort
// ---------------------------------------------------------------------------
__device__ __forceinline__ int atom_cell(const Dev &S, int r, int64_t i,
                                         bool &out) {
  const int32_t *gd = S.grid_dim + 3 * r;
  const double *lo = S.grid_lo + 3 * r;
  int cx = cell_coord(S.x[i], lo[0], S.inv_cell, gd[0], out);
  int cy = cell_coord(S.y[i], lo[1], S.inv_cell, gd[1], out);
  int cz = cell_coord(S.z[i], lo[2], S.inv_cell, gd[2], out);
  return (cz * gd[1] + cy) * gd[0] + cx;
}

// The cell kernels run over the work lists of the step (the tiles, the
// replicas and the cell-sort blocks of the replicas that rebuild): a
// wavefront takes one tile of the list at a time in the per-atom kernels.
__global__ void __launch_bounds__(kBlock) k_cell_count(Dev S) {
  const WorkLists W = work_lists(S);
  const int n = W.count[0];
  const int wv = threadIdx.x / kTile, lane = threadIdx.x & (kTile - 1);
  for (int it = blockIdx.x * (kBlock / kTile) + wv; it < n;
       it += gridDim.x * (kBlock / kTile)) {
    const int tile = W.tiles[it];
    const int64_t i = (int64_t)tile * kTile + lane;
    const int r = S.tile_rep[tile];
    if (S.flag[i] == 3) continue;
    bool out = false;
    const int c = atom_cell(S, r, i, out);
    atomicAdd(&S.cnt[S.cell_off[r] + c], 1);
    if (out) atomicOr(&S.wstatus[r], 4u);
  }
}

// One workgroup per replica of the work list at a time: exclusive scan of
// its cell counts into cell_start; the counters become fill cursors.
__global__ void __launch_bounds__(1024) k_cell_scan(Dev S) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  const WorkLists W = work_lists(S);
  const int nrep = W.count[2];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  for (int it = blockIdx.x; it < nrep; it += gridDim.x) {  // uniform
    const int r = W.reps[it];
    const int64_t c0 = S.cell_off[r], nc = S.cell_off[r + 1] - c0;
    int32_t *start = S.cell_start + c0 + r;
    const int32_t base = (int32_t)S.rep_off[r];
    if (threadIdx.x == 0) carry_s = 0;
    __syncthreads();
    for (int64_t b = 0; b < nc; b += 1024) {
      const int64_t c = b + threadIdx.x;
      const int32_t v = c < nc ? S.cnt[c0 + c] : 0;
      // inclusive wave scan
      int32_t sc = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(sc, o, 64);
        if (lane >= o) sc += t;
      }
      if (lane == 63) wsum[wid] = sc;
      __syncthreads();
      int32_t woff = 0, tot = 0;
      for (int w = 0; w < 16; ++w) {
        if (w < wid) woff += wsum[w];
        tot += wsum[w];
      }
      const int32_t ex = carry_s + woff + sc - v;
      if (c < nc) {
        start[c] = base + ex;
        S.cnt[c0 + c] = base + ex;
      }
      __syncthreads();
      if (threadIdx.x == 0) carry_s += tot;
      __syncthreads();
    }
    if (threadIdx.x == 0) start[nc] = base + carry_s;
  }
}

__global__ void __launch_bounds__(kBlock) k_cell_fill(Dev S) {
  const WorkLists W = work_lists(S);
  const int n = W.count[0];
  const int wv = threadIdx.x / kTile, lane = threadIdx.x & (kTile - 1);
  for (int it = blockIdx.x * (kBlock / kTile) + wv; it < n;
       it += gridDim.x * (kBlock / kTile)) {
    const int tile = W.tiles[it];
    const int64_t i = (int64_t)tile * kTile + lane;
    const int r = S.tile_rep[tile];
    if (S.flag[i] == 3) continue;
    bool out = false;
    const int c = atom_cell(S, r, i, out);
    const int32_t pos = atomicAdd(&S.cnt[S.cell_off[r] + c], 1);
    S.cell_atoms[pos] = (int32_t)i;
  }
}

// Ordering of each cell's slots (the fill order is not deterministic), and
// clearing of its counter for the next build.  Blocks of the cell map take up
// to kSortCells cells of one replica; a wavefront takes kSortCells / 4 of
// them in turn, with the starts of its cells read at once and the next
// cell's slots loaded while a cell is ordered.  A cell of up to 64 atoms is
// ordered by ranks in registers (lane l holds one slot and counts the
// smaller ones, read lane by lane); larger cells by one lane's insertion
// sort.
__global__ void __launch_bounds__(kBlock) k_cell_sort(Dev S) {
  const WorkLists W = work_lists(S);
  const int ncb = W.count[3];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  constexpr int per = kSortCells / (kBlock / kTile);
  int32_t *v = S.cell_atoms;
  for (int it = blockIdx.x; it < ncb; it += gridDim.x) {
    const int4 cb = S.cbmap[W.cblocks[it]];  // replica, first cell, cells
    const int r = cb.x;
    const int nk = min(per, cb.z - w * per);  // this wavefront's cells
    if (nk <= 0) continue;                    // uniform over the wavefront
    const int64_t c0 = S.cell_off[r];
    const int32_t *start = S.cell_start + c0 + r;
    const int cw = cb.y + w * per;
    // lane k <= nk: start of cell cw + k (k = nk: end of the last)
    const int32_t st = start[cw + min(lane, nk)];
    int32_t a = __builtin_amdgcn_readlane(st, 0);
    int32_t e = __builtin_amdgcn_readlane(st, 1);
    int32_t mine = (e - a <= 64 && lane < e - a) ? v[a + lane] : 0x7fffffff;
    for (int k = 0; k < nk; ++k) {
      int32_t an = e, en = e, nxt = 0x7fffffff;
      if (k + 1 < nk) {
        en = __builtin_amdgcn_readlane(st, k + 2);
        if (en - an <= 64 && lane < en - an) nxt = v[an + lane];
      }
      const int32_t n = e - a;
      if (n <= 64) {
        int rank = 0;
        for (int m = 0; m < n; ++m)
          rank += __builtin_amdgcn_readlane(mine, m) < mine ? 1 : 0;
        if (lane < n) v[a + rank] = mine;
      } else if (lane == 0) {
        for (int32_t q = a + 1; q < a + n; ++q) {
          const int32_t key = v[q];
          int32_t m = q - 1;
          while (m >= a && v[m] > key) {
            v[m + 1] = v[m];
            --m;
          }
          v[m + 1] = key;
        }
      }
      if (lane == 0) S.cnt[c0 + cw + k] = 0;
      a = an;
      e = en;
      mine = nxt;
    }
  }
}

// Cell map of the sort: for each replica, blocks of up to kSortCells of its
// cells, replicas in order (one block of 1024 threads; a scan over the
// replicas of their block counts).
__global__ void __launch_bounds__(1024) k_cell_map(Dev S) {
  __shared__ int32_t wsum[16];
  __shared__ int32_t carry_s;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry_s = 0;
  __syncthreads();
  for (int b0 = 0; b0 < S.R; b0 += 1024) {
    const int r = b0 + threadIdx.x;
    const int32_t nc =
        r < S.R ? (int32_t)(S.cell_off[r + 1] - S.cell_off[r]) : 0;
    const int32_t v = (nc + kSortCells - 1) / kSortCells;
    int32_t s = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t t = __shfl_up(s, o, 64);
      if (lane >= o) s += t;
    }
    if (lane == 63) wsum[wid] = s;
    __syncthreads();
    int32_t woff = 0, tot = 0;
    for (int k = 0; k < 16; ++k) {
      if (k < wid) woff += wsum[k];
      tot += wsum[k];
    }
    const int32_t ex = carry_s + woff + s - v;
    for (int k = 0; k < v; ++k)
      S.cbmap[ex + k] = make_int4(r, k * kSortCells,
                                  min(kSortCells, nc - k * kSortCells), 0);
    __syncthreads();
    if (threadIdx.x == 0) carry_s += tot;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// list layout and per-lane LDS rings
// ---------------------------------------------------------------------------
// Verlet and active lists are stored in chunks of 8 entries: entry k of slot
// i is at ((k >> 3) * N + i) * 8 + (k & 7).  A lane reads its next 8 entries
// as 32 contiguous bytes and a wavefront reads 2 KB contiguous at a time.
__device__ __forceinline__ int64_t cl8(int64_t N, int64_t i, int64_t chunk) {
  return (chunk * N + i) << 3;
}

// Value of the unused entries of a lane's last chunk of the Verlet lists
// (nl), and a chunk made of them (read by lanes whose list has ended while
// their wavefront goes on), in global memory so that loads that may read it
// are global loads.
constexpr int32_t kPadEntry = 0x7fffffff;
__device__ __attribute__((aligned(16))) int32_t kPadChunk[8] = {
    kPadEntry, kPadEntry, kPadEntry, kPadEntry,
    kPadEntry, kPadEntry, kPadEntry, kPadEntry};

// The lists the pair passes read (nl_lane) hold byte offsets (j - lo) * 16
// of each neighbour j from the start lo of its block's slot window (the
// union of the windows [lo, hi) of the block's tiles, fixed between list
// builds), so that a block whose window is staged in LDS reads a neighbour
// at the entry itself.  Unused entries hold kPadStaged in blocks whose
// window fits in LDS, which addresses the sentinel after the staged
// positions, and kPadWide in the others; both are at least 16 times the
// window size.
// A block whose window exceeds LDS (a thick wire) may instead stage the
// exact set of its neighbours (gather staging, Dev::gather): the pruning
// kernel lists their offsets from lo in ascending order (Dev::glist, at
// most kStage of them) and writes each entry as 16 times the neighbour's
// rank in that list, with kPadStaged for the unused ones.
// The stage (cap entries, per block: block_stage) and so kPadStaged = 16 cap
// depend on the block's stage class.
constexpr int32_t kPadWide = (int32_t)0xFFFFFFF0u;

__device__ __forceinline__ int32_t pad_staged(int cap) { return cap * 16; }

__device__ __forceinline__ int32_t pad_of_window(int size, int cap) {
  return size > 0 && size <= cap ? pad_staged(cap) : kPadWide;
}

// Entry of neighbour j in a block whose window starts at lo (j >= lo; slot
// counts are below 2^28 in mixed precision, so it fits 32 bits unsigned).
__device__ __forceinline__ int32_t list_entry(int j, int lo) {
  return (int32_t)((uint32_t)(j - lo) << 4);
}

// Per-lane ring of 16 list entries in LDS, interleaved over the STRIDE
// threads of the block (entry e of lane l at e * STRIDE + l, so a
// wavefront's appends hit distinct banks).  Lanes append at their own pace;
// at every 8th step of a wave-uniform loop, each lane holding a full chunk
// writes it to its list as one 32-byte store, so at most 7 + 8 entries are
// ever pending.  Entries past the row's capacity (nch chunks) are counted
// but not stored.
template <int STRIDE>
struct RingT {
  int32_t *lds;  // this lane's first entry
  int cnt;       // entries appended
  int head;      // entries passed on to the list (a multiple of 8)
  __device__ __forceinline__ void push(int j) {
    lds[(cnt & 15) * STRIDE] = j;
    ++cnt;
  }
  // Branch-free append: j is written to the next free slot in any case and
  // counted only when keep holds (an uncounted write is overwritten by the
  // next one).  The slot is never a pending one: at most 15 are pending.
  __device__ __forceinline__ void put(int j, bool keep) {
    lds[(cnt & 15) * STRIDE] = j;
    cnt += keep ? 1 : 0;
  }
  __device__ __forceinline__ void store_chunk(int32_t *list, int64_t N,
                                              int64_t i, int nch) {
    if ((head >> 3) < nch) {
      const int32_t *e = lds + (head & 15) * STRIDE;
      int4 *dst = reinterpret_cast<int4 *>(list + cl8(N, i, head >> 3));
      dst[0] = make_int4(e[0], e[STRIDE], e[2 * STRIDE], e[3 * STRIDE]);
      dst[1] = make_int4(e[4 * STRIDE], e[5 * STRIDE], e[6 * STRIDE],
                         e[7 * STRIDE]);
    }
    head += 8;
  }
  __device__ __forceinline__ void flush(int32_t *list, int64_t N, int64_t i,
                                        int nch) {
    if (cnt - head >= 8) store_chunk(list, N, i, nch);
  }
  // the last chunks; the unused entries of a partial chunk are set to pad
  __device__ __forceinline__ void finish(int32_t *list, int64_t N, int64_t i,
                                         int nch, int32_t pad = kPadEntry) {
    while (cnt > head) {
      for (int e = cnt; e < head + 8; ++e) lds[(e & 15) * STRIDE] = pad;
      store_chunk(list, N, i, nch);
    }
  }
};
using Ring = RingT<kBlock>;

__device__ __forceinline__ bool wave_any(bool p) {
  return __ballot(p) != 0ull;
}

// Loop over the entries k < n of one lane's chunked list starting at chunk
// c0 and moving by dir per chunk; body(j[8], k0) gets the 8 indices of chunk
// c (the atom itself for k >= n, which every pair term excludes).  As in
// chunk_loop_padded below, the next chunk is loaded while body works on the
// current one, into the other of two register sets, and every lane issues
// every load (a lane past its own chunks reads the pad chunk).
template <class F>
__device__ __forceinline__ void chunk_loop(const int32_t *list, int64_t N,
                                           int64_t i, int self, int n,
                                           int64_t c0, int dir, F &&body) {
  const int nmax = __builtin_amdgcn_readfirstlane(wave_max_i(n));
  const int nch = (nmax + 7) >> 3;
  if (nch == 0) return;  // uniform
  const int own = (n + 7) >> 3;
  const int4 *pad = reinterpret_cast<const int4 *>(kPadChunk);
  auto load = [&](int c, int4 &u, int4 &v) {
    const int4 *q =
        c < own ? reinterpret_cast<const int4 *>(
                      list + cl8(N, i, c0 + (int64_t)dir * c))
                : pad;
    u = q[0];
    v = q[1];
    // keeps the loads here (the compiler would sink them to their use)
    asm volatile("" ::: "memory");
  };
  auto run = [&](int c, const int4 &u, const int4 &v) {
    const int k0 = c * 8;
    int j[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 8; ++e) j[e] = k0 + e < n ? j[e] : self;
    body(j, k0);
  };
  int4 a, b, c2, d2;
  load(0, a, b);
  for (int c = 0; c < nch; c += 2) {
    load(min(c + 1, nch - 1), c2, d2);
    run(c, a, b);
    if (c + 1 >= nch) break;  // uniform
    load(min(c + 2, nch - 1), a, b);
    run(c + 1, c2, d2);
  }
}

// A chunk of pad entries addressing the LDS sentinel of the pair passes, in
// global memory (with a constant-memory pointer among the candidates of a
// load, the compiler emits flat loads, which the wavefront must also wait
// for before each LDS read).
// (one per stage class)
constexpr int32_t kPad0 = stage_of_class(0) * 16, kPad1 = stage_of_class(1) * 16;
__device__ __attribute__((aligned(16))) int32_t kPadChunkStaged0[8] = {
    kPad0, kPad0, kPad0, kPad0, kPad0, kPad0, kPad0, kPad0};
__device__ __attribute__((aligned(16))) int32_t kPadChunkStaged1[8] = {
    kPad1, kPad1, kPad1, kPad1, kPad1, kPad1, kPad1, kPad1};
template <int STAGE>
__device__ __forceinline__ const int32_t *pad_chunk_staged() {
  static_assert(STAGE == stage_of_class(0) || STAGE == stage_of_class(1),
                "a stage class");
  return STAGE == stage_of_class(0) ? kPadChunkStaged0 : kPadChunkStaged1;
}

// Loop over the chunks of one lane's list in which every entry may be read:
// the wavefront runs as many chunks as its longest list, a lane past its own
// chunks reads the pad chunk padc, and the unused entries of a lane's last
// chunk hold the same pad value, so body(j[8]) gets 8 entries with no
// per-entry test.  The next chunk is loaded while body works on the current
// one, into the other of two register sets: the loop is unrolled by two, and
// every load is issued by every lane (the prefetch past the last chunk
// reloads the last), so that the compiler's wait counts stay exact and a
// wavefront waits only for the chunk it is about to use.
template <class F>
__device__ __forceinline__ void chunk_loop_padded(const int32_t *list,
                                                  int64_t N, int64_t i, int n,
                                                  const int32_t *padc,
                                                  F &&body) {
  const int nmax = __builtin_amdgcn_readfirstlane(wave_max_i(n));
  const int nch = (nmax + 7) >> 3;
  if (nch == 0) return;  // uniform
  const int own = (n + 7) >> 3;
  const int4 *row = reinterpret_cast<const int4 *>(list + (i << 3));
  const int4 *pad = reinterpret_cast<const int4 *>(padc);
  const int64_t stride = N << 1;  // one chunk, in int4
  auto load = [&](int c, int4 &u, int4 &v) {
    const int4 *q = c < own ? row + c * stride : pad;
    u = q[0];
    v = q[1];
    // keeps the loads here: the compiler would otherwise sink them to their
    // use in the next half, and the wavefront would wait for each chunk
    asm volatile("" ::: "memory");
  };
  auto run = [&](const int4 &u, const int4 &v) {
    const int j[8] = {u.x, u.y, u.z, u.w, v.x, v.y, v.z, v.w};
    body(j);
  };
  int4 a, b, c2, d2;
  load(0, a, b);
  for (int c = 0; c < nch; c += 2) {
    load(min(c + 1, nch - 1), c2, d2);
    run(a, b);
    if (c + 1 >= nch) break;  // uniform
    load(min(c + 2, nch - 1), a, b);
    run(c2, d2);
  }
}

// ---------------------------------------------------------------------------
// Verlet lists
// ---------------------------------------------------------------------------
// One lane per atom.  A replica's lists do not depend on its neighbours in
// the batch, and rows longer than k_cap are truncated and reported.  Two
// ways of producing the candidates:
//  * window scan (mixed precision, k_nlist_mixed): cells are slabs in z, so
//    the cells of the z-slabs around a tile's atoms are one contiguous range
//    of the cell-sorted atom array.  The block copies the positions of that
//    range into LDS once, as FP32 offsets from the tile's first atom, and its
//    wavefronts test the tile's 64 atoms against them (LDS broadcast reads).
//    Taken when the range fits in LDS.
//  * cell scan (otherwise, and in FP64 mode): each lane walks the 27 cells
//    around its own cell, reading candidates from global memory, so that
//    entries come out in ascending cell order (z, y, x), slots ascending
//    within a cell (in mixed precision, within each of the four shares of
//    cells).  Distances are FP64 in FP64 mode, where each lane writes its
//    list through a ring, and exact integer differences of the quantised
//    positions in mixed precision.
// Both give every pair with distance below r_cut + skin (rl); since cells
// are at least rl wide, the extra candidates of the window scan (cells of
// the same slabs outside the 3x3 columns around an atom) are farther away
// than that and never pass the test.  Pairs within a few 1e-6 A of rl may
// fall on either side in the window scan (FP32 offsets); they lie beyond
// r_cut, where every pair term is exactly zero.
// Candidates staged per list-build block (40 KB of LDS).  At 2560 every
// tile of a 10 nm wire in the blocked order fits the box scan (at 1536, one
// in six took the per-lane cell walk); the 512-thread blocks are limited to
// two per CU by registers either way.
constexpr int kCand = 2560;

template <int STRIDE>
struct ListRowT {
  RingT<STRIDE> ring;
  int32_t wlo, whi;  // slot window of the row
  __device__ __forceinline__ void add(int32_t j) {
    ring.push(j);
    wlo = min(wlo, j);
    whi = max(whi, j);
  }
};

// FP64 cell scan: this lane's atom against the atoms of the 27 cells around
// its cell, in cell order (FP64 distances); entries go to the lane's ring.
template <class Row>
__device__ __forceinline__ void nlist_cells(const Dev &S, int64_t i, int r,
                                            bool real, int cx, int cy, int cz,
                                            double rl2, int nch, Row &row) {
  const int64_t N = S.N;
  const int32_t *gd = S.grid_dim + 3 * r;
  const int32_t *start = S.cell_start + S.cell_off[r] + r;
  const double xi = S.x[i], yi = S.y[i], zi = S.z[i];
  int cc = -1;
  int32_t s = 0, e = 0;
  bool live = real;
  for (int it = 0;; ++it) {
    if (live) {
      while (s >= e) {
        if (++cc >= 27) {
          live = false;
          break;
        }
        const int kz = cz + cc / 9 - 1, ky = cy + (cc / 3) % 3 - 1,
                  kx = cx + cc % 3 - 1;
        if (kx >= 0 && kx < gd[0] && ky >= 0 && ky < gd[1] && kz >= 0 &&
            kz < gd[2]) {
          const int c = (kz * gd[1] + ky) * gd[0] + kx;
          s = start[c];
          e = start[c + 1];
        }
      }
    }
    if (!wave_any(live)) break;
    if (live) {
      const int32_t j = S.cell_atoms[s++];
      if (j != (int32_t)i) {
        const double dx = S.x[j] - xi, dy = S.y[j] - yi, dz = S.z[j] - zi;
        if (dx * dx + dy * dy + dz * dz < rl2) row.add(j);
      }
    }
    if ((it & 7) == 7) row.ring.flush(S.nl, N, i, nch);
  }
}

// Mixed-precision cell scan, for tiles whose slabs exceed LDS: this lane's
// atom against the atoms of cells q, q + nq, q + 2 nq, ... of the 27 around
// its cell (nq wavefronts share the scan), reading candidate positions from
// global memory; near(j, d2, -1) is called for each candidate j within the
// list radius, with its squared distance d2 (exact integer differences of
// the quantised positions, quanta^2), in cell order.  A lane takes up to 4
// candidates of its current cell at a time, so that their slot and position
// loads are in flight together.
template <class F>
__device__ __forceinline__ void cells_scan(const Dev &S, int64_t i, int r,
                                           bool real, int cx, int cy, int cz,
                                           int4 qi, float rl2q, int q, int nq,
                                           F &&near) {
  const int32_t *gd = S.grid_dim + 3 * r;
  const int32_t *start = S.cell_start + S.cell_off[r] + r;
  int cc = q - nq;
  int32_t s = 0, e = 0;
  bool live = real;
  for (;;) {
    if (live) {
      while (s >= e) {
        cc += nq;
        if (cc >= 27) {
          live = false;
          break;
        }
        const int kz = cz + cc / 9 - 1, ky = cy + (cc / 3) % 3 - 1,
                  kx = cx + cc % 3 - 1;
        if (kx >= 0 && kx < gd[0] && ky >= 0 && ky < gd[1] && kz >= 0 &&
            kz < gd[2]) {
          const int c = (kz * gd[1] + ky) * gd[0] + kx;
          s = start[c];
          e = start[c + 1];
        }
      }
    }
    if (!wave_any(live)) break;
    if (live) {
      const int nb = min(4, e - s);
      int32_t jj[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) jj[k] = k < nb ? S.cell_atoms[s + k] : -1;
      int4 qq[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        qq[k] = jj[k] >= 0 ? S.qpos[jj[k]] : make_int4(0, 0, 0, 0);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        if (jj[k] < 0 || jj[k] == (int32_t)i) continue;
        const float dx = (float)(qq[k].x - qi.x);
        const float dy = (float)(qq[k].y - qi.y);
        const float dz = (float)(qq[k].z - qi.z);
        const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
        if (d2 < rl2q) near(jj[k], d2, -1);
      }
      s += nb;
    }
  }
}

// Tests this lane's atom (FP32 offset pi from the block origin) against
// window candidates [a, b) of cand (x, y, z offsets and the slot as bits;
// a and b uniform over the wavefront) and calls near(j, d2, t) for each
// candidate t, of slot j, within the list radius, with its squared distance
// d2 (quanta^2), in candidate order.  Candidates are read in
// groups of 8, and this wavefront takes groups q, q + nq, q + 2 nq, ... of
// the range (nq wavefronts share the scan of one tile).  cand holds 8
// filler entries past the window so the last group stays in bounds, and
// entries at b or beyond are never taken.
template <class F>
__device__ __forceinline__ void window_scan(int64_t i, bool real, float4 pi,
                                            const float4 *cand, int a, int b,
                                            float rl2q, int q, int nq,
                                            F &&near) {
  const int32_t self = real ? (int32_t)i : -2;
  a = __builtin_amdgcn_readfirstlane(a);
  b = __builtin_amdgcn_readfirstlane(b);
  for (int t0 = a + 8 * q; t0 < b; t0 += 8 * nq) {
    float4 c[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) c[e] = cand[t0 + e];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float dx = c[e].x - pi.x;
      const float dy = c[e].y - pi.y;
      const float dz = c[e].z - pi.z;
      const int32_t j = __float_as_int(c[e].w);
      const float d2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
      if (d2 < rl2q && j != self && t0 + e < b && real) near(j, d2, t0 + e);
    }
  }
}

// Lane order of the pair passes: the block's atoms by descending list
// length, ties by slot (keys are distinct).  key[t] is set by every thread
// t < kBlock; returns this thread's rank among the block's nt tiles.
__device__ __forceinline__ int lane_rank(const int32_t *key, int t, int nt) {
  const int32_t k = key[t];
  int rank = 0;
  for (int m = 0; m < nt * kTile; ++m) rank += key[m] < k ? 1 : 0;
  return rank;
}
__device__ __forceinline__ int32_t lane_key(int nn_i, int t) {
  return nn_i < 0 ? 0x7fffffff : ((255 - min(nn_i, 255)) << 8) | t;
}

// FP64 list build: one lane per atom, the 27-cell walk with FP64 distances.
__global__ void __launch_bounds__(kBlock) k_nlist_fp64(Dev S, double rl2) {
  __shared__ int32_t ring_lds[16 * kBlock];
  __shared__ int32_t key[kBlock];
  const int tid = threadIdx.x, w = tid / kTile;
  const int2 bm = S.bmap[blockIdx.x];  // first tile, tiles (1..4)
  const int r = S.tile_rep[bm.x];
  if (!rebuilds(S, r)) return;  // uniform over the block
  const bool valid = w < bm.y;
  const int64_t i = ((int64_t)bm.x + w) * kTile + (tid & (kTile - 1));
  int nn_i = -1;  // list length of this thread's atom (-1: no atom)
  if (valid) {
    const bool real = S.flag[i] != 3;
    const int32_t *gd = S.grid_dim + 3 * r;
    const double *lo = S.grid_lo + 3 * r;
    bool out = false;
    const int cx = cell_coord(S.x[i], lo[0], S.inv_cell, gd[0], out);
    const int cy = cell_coord(S.y[i], lo[1], S.inv_cell, gd[1], out);
    const int cz = cell_coord(S.z[i], lo[2], S.inv_cell, gd[2], out);
    const int64_t N = S.N;
    const int nch = S.k_cap >> 3;
    ListRowT<kBlock> row{Ring{ring_lds + tid, 0, 0}, (int32_t)i, (int32_t)i};
    nlist_cells(S, i, r, real, cx, cy, cz, rl2, nch, row);
    row.ring.finish(S.nl, N, i, nch);
    const int32_t wlo = -wave_max_i(-row.wlo);
    const int32_t whi = wave_max_i(row.whi);
    if ((tid & 63) == 0) S.win[i / kTile] = make_int2(wlo, whi + 1);
    const int total = row.ring.cnt;
    if (total > S.k_cap) {
      atomicMax(S.nnmax, total);
      atomicOr(&S.wstatus[r], 1u);
    }
    nn_i = real ? min(total, S.k_cap) : 0;
    S.nn[i] = nn_i;
    S.xr[i] = S.x[i];
    S.yr[i] = S.y[i];
    S.zr[i] = S.z[i];
  }
  key[tid] = lane_key(nn_i, tid);
  __syncthreads();
  if (valid) {
    const int rank = lane_rank(key, tid, bm.y);
    S.lane_atom[(int64_t)bm.x * kTile + rank] = (uint8_t)tid;
    S.atom_lane[i] = (uint8_t)rank;
  }
}

// The runs first, first + 1, ..., first + cnt - 1 at dst[off], ... of every
// lane of the wavefront, one run at a time over the whole wavefront.  Only
// the replicas that rebuild or prune add entries, so most wavefronts have
// few runs or none.
__device__ __forceinline__ void write_runs(int32_t *dst, int32_t first,
                                           int32_t cnt, int32_t off,
                                           int lane) {
  uint64_t m = __ballot(cnt > 0);
  while (m) {  // uniform
    const int l = __builtin_ctzll(m);
    m &= m - 1;
    const int32_t f = __shfl(first, l, 64), c = __shfl(cnt, l, 64),
                  o = __shfl(off, l, 64);
    for (int x = lane; x < c; x += 64) dst[o + x] = f + x;
  }
}

// The work lists of the step (WorkLists) from the rebuild and pruning flags
// of every replica.  One block of 1024 threads; a scan over the replicas of
// the entries each adds to each list, and of its blocks in the list-build
// and cell-sort maps (replicas in order there too).
__global__ void __launch_bounds__(1024) k_worklist(Dev S) {
  // scanned per replica: tiles, list-build blocks and cell-sort blocks
  // listed, replica listed; its blocks in the two maps
  constexpr int kL = 6;
  __shared__ int32_t wsum[kL][16];
  __shared__ int32_t carry[kL], tot[kL];
  const WorkLists W = work_lists(S);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  if (tid < kL) carry[tid] = 0;
  __syncthreads();
  for (int b0 = 0; b0 < S.R; b0 += 1024) {
    const int r = b0 + tid;
    int32_t t0 = 0, nt = 0, nc = 0;
    bool reb = false, upd = false;
    if (r < S.R) {
      t0 = (int32_t)(S.rep_off[r] / kTile);
      nt = (int32_t)(S.rep_off[r + 1] / kTile) - t0;
      nc = (int32_t)(S.cell_off[r + 1] - S.cell_off[r]);
      reb = rebuilds(S, r);
      upd = reb || prunes(S, r);
    }
    if (S.rstatus != nullptr) {
      // step loops: replicas rebuilt, and pruned without a rebuild
      const unsigned long long br = __ballot(reb), bp = __ballot(upd && !reb);
      if (lane == 0 && (br | bp)) {
        unsigned long long *ctr = reinterpret_cast<unsigned long long *>(
            S.callb + kCallRebuilds);
        atomicAdd(ctr, (unsigned long long)__popcll(br));
        atomicAdd(ctr + 1, (unsigned long long)__popcll(bp));
      }
    }
    const int tpb = r < S.R ? shape_tpb(rep_shape(S, r)) : 4;
    const int32_t nb = (nt + tpb - 1) / tpb;
    const int32_t ncb = (nc + kSortCells - 1) / kSortCells;
    const int32_t v[kL] = {reb ? nt : 0, upd ? nb : 0, reb ? ncb : 0,
                           reb ? 1 : 0,  nb,          ncb};
    int32_t sc[kL];
#pragma unroll
    for (int k = 0; k < kL; ++k) {
      int32_t x = v[k];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
      }
      sc[k] = x;
      if (lane == 63) wsum[k][wid] = x;
    }
    __syncthreads();
    // wave totals -> exclusive wave offsets (in place) and chunk totals
    if (tid < kL) {
      int32_t acc = 0;
      for (int m = 0; m < 16; ++m) {
        const int32_t t = wsum[tid][m];
        wsum[tid][m] = acc;
        acc += t;
      }
      tot[tid] = acc;
    }
    __syncthreads();
    int32_t ex[kL];
#pragma unroll
    for (int k = 0; k < kL; ++k) ex[k] = carry[k] + wsum[k][wid] + sc[k] - v[k];
    if (reb) W.reps[ex[3]] = r;
    // each wavefront writes the runs of its own replicas
    write_runs(W.tiles, t0, v[0], ex[0], lane);
    write_runs(W.blocks, r < S.R ? S.boff[r] : 0, v[1], ex[1], lane);
    write_runs(W.cblocks, ex[5], v[2], ex[2], lane);
    __syncthreads();
    if (tid < kL) carry[tid] += tot[tid];
    __syncthreads();
  }
  // counts: tiles, list-build blocks, replicas, cell-sort blocks
  if (tid == 0) {
    W.count[0] = carry[0];
    W.count[1] = carry[1];
    W.count[2] = carry[3];
    W.count[3] = carry[2];
  }
}

// Exclusive block-wide prefix of v over the NT threads (every thread takes
// part); *total gets the sum.  wsum: NT / 64 ints of LDS.
template <int NT = kBlock>
__device__ __forceinline__ int block_excl_scan(int v, int32_t *wsum,
                                               int *total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(x, o, 64);
    if (lane >= o) x += t;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int before = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    const int t = wsum[k];
    before += k < w ? t : 0;
    tot += t;
  }
  __syncthreads();  // wsum may be reused
  *total = tot;
  return before + x - v;
}

// Mixed-precision list build, one tile per block and work item (the tiles
// of the work list).  The block's kNlWaves wavefronts share the scan of
// the tile's candidates, the cell-sorted atoms of the z-slabs around its
// atoms: wavefront q takes every kNlWaves-th group of 8.  So the rebuild of
// a single replica, which would leave most of the GPU idle, spreads over
// every compute unit and is not bound by one wavefront's walk over the
// ~1000 candidates.  The scan runs twice: the first pass counts each
// share's pairs, the second writes them at their final entries, share q
// after shares 0..q-1.  A row is thus the pairs in candidate order within
// each share, shares in order, whatever the timing: first the pairs within
// the core radius (Dev::core_r2q; their number in ncore), then the others,
// each part so ordered.  When the slabs exceed
// LDS, the wavefronts share the walk over the 27 cells around each atom the
// same way (wavefront q takes cells q, q + kNlWaves, ...).  The
// lane-ordered, pruned rows are made by the pruning kernel.
// Threads of a list-build block: eight wavefronts share the scan of one
// tile (a single replica's rebuild runs about one such block per CU, and
// eight shares halve each wavefront's serial walk against four; sixteen
// were slower).
constexpr int kNlBlock = 512;
constexpr int kNlWaves = kNlBlock / kTile;
// Pairs per row and share that the list build's counting scan keeps for its
// writing pass (a share of a 3 nm wire's row averages about 15).
constexpr int kFound = 32;
static_assert(kCand + 8 <= 0x8000, "candidate indices fit in 15 bits");

constexpr int kBoxRows = 64;  // rows of cells of the box scan, at most

__global__ void __launch_bounds__(kNlBlock) k_nlist_mixed(Dev S, float rl2q) {
  __shared__ float4 cand[kCand + 8];
  __shared__ int32_t qcnt[kNlWaves][kTile];
  __shared__ uint16_t found[kNlWaves][kFound][kTile];
  __shared__ int32_t qcore[kNlWaves][kTile];
  __shared__ int2 qwin[kNlWaves];
  __shared__ int32_t rowbeg[kBoxRows], rowlen[kBoxRows], rowpre[kBoxRows + 1];
  __shared__ int32_t wsum[kNlBlock / 64];
  const int tid = threadIdx.x;
  const int q = tid / kTile;  // share of the candidate scan
  const int lane = tid & (kTile - 1);
  const WorkLists W = work_lists(S);
  const int ntl = W.count[0];
  const int32_t *tiles = W.tiles;
  const int64_t N = S.N;
  for (int it = blockIdx.x; it < ntl; it += gridDim.x) {  // uniform
    const int tile = tiles[it];
    const int r = S.tile_rep[tile];
    const int64_t i = (int64_t)tile * kTile + lane;
    const bool real = S.flag[i] != 3;
    const int32_t *gd = S.grid_dim + 3 * r;
    const double *lo = S.grid_lo + 3 * r;
    bool out = false;
    const int cx = cell_coord(S.x[i], lo[0], S.inv_cell, gd[0], out);
    const int cy = cell_coord(S.y[i], lo[1], S.inv_cell, gd[1], out);
    const int cz = cell_coord(S.z[i], lo[2], S.inv_cell, gd[2], out);
    const int4 qi = S.qpos[i];
    // z-cell range of the tile's real atoms (empty: lo > hi); the same in
    // every wavefront of the block
    const int zlo = -wave_max_i(real ? -cz : -0x7fffffff);
    const int zhi = wave_max_i(real ? cz : -1);
    bool window = false;  // uniform over the block
    int m = 0;
    float4 pi = make_float4(0.f, 0.f, 0.f, 0.f);
    if (zlo <= zhi) {
      const int gxy = gd[0] * gd[1];
      const int32_t *start = S.cell_start + S.cell_off[r] + r;
      const int32_t s0 = start[max(zlo - 1, 0) * gxy];
      const int32_t s1 = start[(min(zhi + 1, gd[2] - 1) + 1) * gxy];
      m = s1 - s0;
      window = m <= kCand;
      if (window) {
        const int4 o = S.qpos[(int64_t)tile * kTile];
        // all of a thread's slot reads, then all of its position reads (m is
        // uniform, so are the trip counts)
        constexpr int kPer = (kCand + 8 + kNlBlock - 1) / kNlBlock;
        int32_t jj[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
          const int t = tid + k * kNlBlock;
          jj[k] = t < m ? S.cell_atoms[s0 + t] : -1;
        }
        int4 qq[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k)
          qq[k] = jj[k] >= 0 ? S.qpos[jj[k]] : make_int4(0, 0, 0, 0);
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
          const int t = tid + k * kNlBlock;
          if (t < m + 8)
            cand[t] = jj[k] >= 0
                          ? make_float4((float)(qq[k].x - o.x),
                                        (float)(qq[k].y - o.y),
                                        (float)(qq[k].z - o.z),
                                        __int_as_float(jj[k]))
                          : make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
        }
        pi = make_float4((float)(qi.x - o.x), (float)(qi.y - o.y),
                         (float)(qi.z - o.z), 0.f);
      } else {
        // slabs too wide (thick wires): the cells around the tile's cell box,
        // one range of cell_atoms per row of cells along x, keeping the
        // candidates within the list radius of the box of the tile's
        // quantised positions (a superset of every atom's neighbours), in
        // row order (z, then y), compacted by a block-wide scan
        const int xlo = -wave_max_i(real ? -cx : -0x7fffffff);
        const int xhi = wave_max_i(real ? cx : -1);
        const int ylo = -wave_max_i(real ? -cy : -0x7fffffff);
        const int yhi = wave_max_i(real ? cy : -1);
        const int x0 = max(xlo - 1, 0), x1 = min(xhi + 1, gd[0] - 1);
        const int y0 = max(ylo - 1, 0), y1 = min(yhi + 1, gd[1] - 1);
        const int z0 = max(zlo - 1, 0), z1 = min(zhi + 1, gd[2] - 1);
        const int ny = y1 - y0 + 1, nrow = ny * (z1 - z0 + 1);
        if (nrow <= kBoxRows) {
          if (tid < nrow) {
            const int c = ((z0 + tid / ny) * gd[1] + y0 + tid % ny) * gd[0];
            rowbeg[tid] = start[c + x0];
            rowlen[tid] = start[c + x1 + 1] - start[c + x0];
          }
          __syncthreads();
          if (tid == 0) {
            int acc = 0;
            for (int k = 0; k < nrow; ++k) {
              rowpre[k] = acc;
              acc += rowlen[k];
            }
            rowpre[nrow] = acc;
          }
          __syncthreads();
          const int total = rowpre[nrow];
          // the tile's box in quanta (the same in every wavefront)
          const int bx0 = -wave_max_i(real ? -qi.x : -0x7fffffff);
          const int bx1 = wave_max_i(real ? qi.x : -0x7fffffff);
          const int by0 = -wave_max_i(real ? -qi.y : -0x7fffffff);
          const int by1 = wave_max_i(real ? qi.y : -0x7fffffff);
          const int bz0 = -wave_max_i(real ? -qi.z : -0x7fffffff);
          const int bz1 = wave_max_i(real ? qi.z : -0x7fffffff);
          const int4 o = S.qpos[(int64_t)tile * kTile];
          int kept = 0;
          for (int t0 = 0; t0 < total; t0 += kNlBlock) {  // uniform
            const int t = t0 + tid;
            bool keep = false;
            float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
            if (t < total) {
              // the row of candidate t: the last row that starts at or
              // before it (rowpre is non-decreasing), by bisection
              int k = 0, kh = nrow - 1;
              while (k < kh) {
                const int mid = (k + kh + 1) >> 1;
                if (rowpre[mid] <= t)
                  k = mid;
                else
                  kh = mid - 1;
              }
              const int32_t j = S.cell_atoms[rowbeg[k] + (t - rowpre[k])];
              const int4 qj = S.qpos[j];
              const float ex = (float)max(max(bx0 - qj.x, qj.x - bx1), 0);
              const float ey = (float)max(max(by0 - qj.y, qj.y - by1), 0);
              const float ez = (float)max(max(bz0 - qj.z, qj.z - bz1), 0);
              keep = fmaf(ex, ex, fmaf(ey, ey, ez * ez)) < rl2q;
              c = make_float4((float)(qj.x - o.x), (float)(qj.y - o.y),
                              (float)(qj.z - o.z), __int_as_float(j));
            }
            int n_kept = 0;
            const int pos = kept + block_excl_scan<kNlBlock>(keep ? 1 : 0, wsum, &n_kept);
            if (keep && pos < kCand) cand[pos] = c;
            kept += n_kept;
          }
          if (kept <= kCand) {
            window = true;
            m = kept;
            if (tid < 8)
              cand[m + tid] = make_float4(0.f, 0.f, 0.f, __int_as_float(-1));
            pi = make_float4((float)(qi.x - o.x), (float)(qi.y - o.y),
                             (float)(qi.z - o.z), 0.f);
          }
        }
      }
    }
    __syncthreads();
    int cnt = 0, cnt_c = 0;  // pairs of this share, of them in the core
    int32_t wlo = (int32_t)i, whi = (int32_t)i;  // slot window of the row
    const float core2 = S.core_r2q;
    // from window candidates, the first kFound pairs of the share are also
    // kept (candidate index, core flag in the top bit) for the writing pass
    auto count = [&](int32_t j, float d2, int t) {
      const bool c = d2 < core2;
      if (cnt < kFound)
        found[q][cnt][lane] = (uint16_t)(t | (c ? 0x8000 : 0));
      ++cnt;
      cnt_c += c ? 1 : 0;
      wlo = min(wlo, j);
      whi = max(whi, j);
    };
    if (window)
      window_scan(i, real, pi, cand, 0, m, rl2q, q, kNlWaves, count);
    else
      cells_scan(S, i, r, real, cx, cy, cz, qi, rl2q, q, kNlWaves, count);
    qcnt[q][lane] = cnt;
    qcore[q][lane] = cnt_c;
    const int32_t wl = -wave_max_i(-wlo);
    const int32_t wh = wave_max_i(whi);
    if (lane == 0) qwin[q] = make_int2(wl, wh);
    __syncthreads();
    // entries of all shares and of shares 0..q-1, in all and in the core:
    // the row holds the core pairs of every share first, then the others
    int total = 0, before = 0, total_c = 0, before_c = 0;
#pragma unroll
    for (int k = 0; k < kNlWaves; ++k) {
      const int c = qcnt[k][lane], cc = qcore[k][lane];
      before += k < q ? c : 0;
      total += c;
      before_c += k < q ? cc : 0;
      total_c += cc;
    }
    int ec = before_c, es = total_c + before - before_c;
    auto write = [&](int32_t j, float d2, int) {
      const int e = d2 < core2 ? ec++ : es++;
      if (e < S.k_cap) S.nl[cl8(N, i, e >> 3) + (e & 7)] = j;
    };
    // the kept pairs when every share of every row fitted (uniform), else a
    // second scan; either writes the same entries in the same order
    if (window && !__syncthreads_or(cnt > kFound)) {
      for (int k = 0; k < cnt; ++k) {
        const uint32_t f = found[q][k][lane];
        const int32_t j = __float_as_int(cand[f & 0x7fffu].w);
        const int e = (f & 0x8000u) ? ec++ : es++;
        if (e < S.k_cap) S.nl[cl8(N, i, e >> 3) + (e & 7)] = j;
      }
    } else if (window) {
      window_scan(i, real, pi, cand, 0, m, rl2q, q, kNlWaves, write);
    } else {
      cells_scan(S, i, r, real, cx, cy, cz, qi, rl2q, q, kNlWaves, write);
    }
    // the unused entries of the row's last chunk
    if (q == kNlWaves - 1 && total < S.k_cap)
      for (int f = total; f < ((total + 7) & ~7); ++f)
        S.nl[cl8(N, i, f >> 3) + (f & 7)] = kPadEntry;
    if (q == 0) {
      if (total > S.k_cap) {
        atomicMax(S.nnmax, total);
        atomicOr(&S.wstatus[r], 1u);
      }
      S.nn[i] = real ? min(total, S.k_cap) : 0;
      S.ncore[i] = real ? min(total_c, S.k_cap) : 0;
      S.xr[i] = S.x[i];
      S.yr[i] = S.y[i];
      S.zr[i] = S.z[i];
    }
    // slot window [lo, hi) of the tile's rows: read by the pair passes to
    // stage neighbour positions in LDS
    if (tid == 0) {
      int2 tw = qwin[0];
#pragma unroll
      for (int k = 1; k < kNlWaves; ++k) {
        tw.x = min(tw.x, qwin[k].x);
        tw.y = max(tw.y, qwin[k].y);
      }
      S.win[tile] = make_int2(tw.x, tw.y + 1);
    }
    __syncthreads();  // cand, qcnt and qwin serve the next tile
  }
}

// Block map of the list build and the pair passes: for each replica, blocks
// of up to tpb of its tiles (its launch shape), replicas in order within each
// stage class, the classes one after another from cls_off[c]; boff[r] is the
// replica's first block.  One block of 1024 threads; a scan over the
// replicas of their block counts per class.
__global__ void __launch_bounds__(1024) k_block_map(Dev S) {
  __shared__ int32_t wsum[kStageClasses][16];
  __shared__ int32_t carry_s[kStageClasses];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (threadIdx.x < kStageClasses) carry_s[threadIdx.x] = 0;
  __syncthreads();
  for (int b0 = 0; b0 < S.R; b0 += 1024) {
    const int r = b0 + threadIdx.x;
    int32_t t0 = 0, nt = 0, tpb = 4, cls = 0;
    if (r < S.R) {
      t0 = (int32_t)(S.rep_off[r] / kTile);
      nt = (int32_t)(S.rep_off[r + 1] / kTile) - t0;
      const int32_t sh = rep_shape(S, r);
      tpb = shape_tpb(sh);
      cls = shape_cls(sh);
    }
    const int32_t v = (nt + tpb - 1) / tpb;
    int32_t ex[kStageClasses], tot[kStageClasses];
#pragma unroll
    for (int c = 0; c < kStageClasses; ++c) {
      const int32_t vc = cls == c ? v : 0;
      int32_t sc = vc;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int32_t t = __shfl_up(sc, o, 64);
        if (lane >= o) sc += t;
      }
      if (lane == 63) wsum[c][wid] = sc;
      ex[c] = sc - vc;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < kStageClasses; ++c) {
      int32_t woff = 0, t = 0;
      for (int k = 0; k < 16; ++k) {
        if (k < wid) woff += wsum[c][k];
        t += wsum[c][k];
      }
      ex[c] += carry_s[c] + woff + S.cls_off[c];
      tot[c] = t;
    }
    if (r < S.R) {
      const int32_t first = ex[cls];
      S.boff[r] = first;
      for (int k = 0; k < v; ++k)
        S.bmap[first + k] = make_int2(t0 + tpb * k, min(tpb, nt - tpb * k));
    }
    __syncthreads();
    if (threadIdx.x < kStageClasses) carry_s[threadIdx.x] += tot[threadIdx.x];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// pass 1: density rho_i -> g_i = 1/sqrt(rho_i)
// ---------------------------------------------------------------------------
// Keeps a loop-invariant value in a VGPR (a VOP3 instruction reads at most
// one scalar operand, so two uniform constants would otherwise be copied
// into VGPRs on every iteration).
template <class T>
__device__ __forceinline__ T in_vgpr(T v) {
  asm volatile("" : "+v"(v));
  return v;
}

// Gather of one quantised position by a 32-bit byte offset from a uniform
// base (slot counts are below 2^28 in mixed precision).
__device__ __forceinline__ int4 gather_q(const int4 *qp, int j) {
  return *reinterpret_cast<const int4 *>(reinterpret_cast<const char *>(qp) +
                                         ((uint32_t)j << 4));
}

// The pair passes run over the blocks of the list build (up to four tiles of
// one replica).  Lane p of a block evaluates atom b0 + lane_atom[b0 + p]: the
// list build orders each block's atoms by descending list length, so that the
// lists of a wavefront have similar lengths (a wavefront runs as many steps as
// its longest list).  Each atom's own sums run in list order whichever lane
// takes it, so results do not depend on the assignment.
struct PairBlock {
  int64_t blk; // index in the block map
  int64_t b0;  // first slot
  int t0, nt;  // first tile, tiles
  int p;       // this thread's position
  bool valid;  // p < 64 nt
  int64_t i;   // the atom this thread evaluates
  int n;       // its list length; its list is row b0 + p of nl_lane
};

// base: first block-map index of this launch (its stage class).
__device__ __forceinline__ PairBlock pair_block(const Dev &S, int base) {
  PairBlock B;
  B.blk = base + xcd_block();
  const int2 bm = S.bmap[B.blk];
  B.t0 = bm.x;
  B.nt = bm.y;
  B.b0 = (int64_t)bm.x * kTile;
  B.p = threadIdx.x;
  B.valid = B.p < bm.y * kTile;
  B.i = B.b0 + (B.valid ? (int)S.lane_atom[B.b0 + B.p] : 0);
  B.n = B.valid ? S.nn_lane[B.b0 + B.p] : 0;
  return B;
}

// Neighbour positions are gathered from LDS when the block's neighbours fit:
// atoms are ordered along the wire, so the neighbours of a block's slots lie
// in a short slot window [lo, hi) recorded per tile by the list build; the
// block copies qpos[lo, hi) into LDS with coalesced loads and gathers from
// there.  Blocks with wider windows (thick wires) gather from global memory.
// Slot window of the block (union over its tiles); size 0 when some tile has
// no list yet.
__device__ __forceinline__ void block_window(const Dev &S, const PairBlock &B,
                                             int &lo, int &size) {
  int l = 0x7fffffff, h = 0;
  bool ok = true;
#pragma unroll
  for (int t = 0; t < kBlock / kTile; ++t) {
    if (t < B.nt) {
      const int2 w = S.win[B.t0 + t];
      ok = ok && w.y > w.x;
      l = min(l, w.x);
      h = max(h, w.y);
    }
  }
  lo = l;
  size = ok ? h - l : 0;
}

// Copies qpos[lo, lo+size) to lq[0, size) (all threads of the block take
// part) and puts at lq[kStage] a sentinel position for the unused list
// entries, which then contribute exactly nothing: their distance is beyond
// r_cut, where the tail expressions vanish.  The sentinel lies 2^30 quanta
// along x from the block's first atom; it is used only when every atom of
// the block lies within 2^29 quanta of that atom along x, so it is at least
// 2^29 quanta (32 A at 24 bits) from each of them and no difference
// overflows.  Returns that condition (uniform over the block).
// The sentinel and the condition for it, after the block has copied its
// staged positions (all threads of the block take part).
__device__ __forceinline__ bool stage_sentinel(const Dev &S, int4 *lq,
                                               const PairBlock &B, int cap) {
  const int4 q0 = S.qpos[B.b0];
  const int xi = B.valid ? S.qpos[B.b0 + B.p].x : q0.x;
  const int64_t d = (int64_t)xi - (int64_t)q0.x;
  const bool near = d > -(1ll << 29) && d < (1ll << 29);
  if (threadIdx.x == 0)
    lq[cap] = make_int4(q0.x >= 0 ? q0.x - (1 << 30) : q0.x + (1 << 30),
                           q0.y, q0.z, 0);
  return __syncthreads_and(near) != 0;
}

__device__ __forceinline__ bool stage(const Dev &S, int4 *lq,
                                      const PairBlock &B, int lo, int size,
                                      int cap) {
  for (int t = threadIdx.x; t < size; t += kBlock) lq[t] = S.qpos[lo + t];
  return stage_sentinel(S, lq, B, cap);
}

// Gather staging: lq[k] = qpos[lo + glist[k]] for the gc listed neighbours
// of the block, then the sentinel as above.
__device__ __forceinline__ bool stage_gather(const Dev &S, int4 *lq,
                                             const PairBlock &B, int lo,
                                             int gc, int cap) {
  // all of a thread's list reads, then all of its position reads (each
  // position read depends on a list read; gc <= kStage)
  const uint16_t *g = S.glist + B.blk * kStage;
  constexpr int kPer = (kStage + kBlock - 1) / kBlock;
  int off[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int t = threadIdx.x + k * kBlock;
    off[k] = t < gc ? (int)g[t] : 0;
  }
  int4 v[kPer];
#pragma unroll
  for (int k = 0; k < kPer; ++k) v[k] = S.qpos[lo + off[k]];
#pragma unroll
  for (int k = 0; k < kPer; ++k) {
    const int t = threadIdx.x + k * kBlock;
    if (t < gc) lq[t] = v[k];
  }
  return stage_sentinel(S, lq, B, cap);
}

// LDS entry of list entry j: lq[min(j, lo + cap) - lo] (kPadEntry -> the
// sentinel), with the byte offset formed as min(j, jmax) * 16 - lo * 16.
struct StagedIndex {
  int jmax;       // lo + cap
  uint32_t nlo;   // -lo * 16 (mod 2^32)
  __device__ __forceinline__ StagedIndex(int lo, int cap)
      : jmax(lo + cap), nlo(0u - ((uint32_t)lo << 4)) {}
  __device__ __forceinline__ int4 get(const int4 *lq, int j) const {
    const uint32_t off = ((uint32_t)min(j, jmax) << 4) + nlo;
    return *reinterpret_cast<const int4 *>(
        reinterpret_cast<const char *>(lq) + off);
  }
};

// Staged position at byte offset e of lq (an entry of nl_lane).
__device__ __forceinline__ int4 lds_at(const int4 *lq, int32_t e) {
  return *reinterpret_cast<const int4 *>(reinterpret_cast<const char *>(lq) +
                                         (uint32_t)e);
}

// Slot of an entry of nl_lane in a block that is not staged: lo + e/16, or
// self for a pad entry (self then adds nothing: its distance is 0).
struct ListDecode {
  int lo;
  uint32_t lim;  // 16 * window size; pad entries are at least this
  int self;
  __device__ __forceinline__ ListDecode(int lo_, int size, int self_)
      : lo(size > 0 ? lo_ : 0), lim((uint32_t)size << 4), self(self_) {}
  __device__ __forceinline__ int operator()(int32_t e) const {
    return (uint32_t)e < lim ? lo + (int)((uint32_t)e >> 4) : self;
  }
};

// The same for a block whose entries are ranks in its gather list (gather
// staging taken at pruning, but the sentinel condition failed at this pass).
struct GatherDecode {
  int lo;
  const uint16_t *g;
  uint32_t lim;  // 16 * listed neighbours
  int self;
  __device__ __forceinline__ GatherDecode(const Dev &S, const PairBlock &B,
                                          int lo_, int gc, int self_)
      : lo(lo_), g(S.glist + B.blk * kStage), lim((uint32_t)gc << 4),
        self(self_) {}
  __device__ __forceinline__ int operator()(int32_t e) const {
    return (uint32_t)e < lim ? lo + (int)g[(uint32_t)e >> 4] : self;
  }
};

// Lane-ordered, pruned rows (nl_lane) of the list-build blocks of the work
// list: blocks of replicas whose lists were just rebuilt, which first take
// their lane order from the new list lengths, and of replicas in which some
// atom has moved more than the pruning half-width since their lists were
// last pruned.  Lanes take the block's atoms in slot order, so the full
// rows are read coalesced; each lane writes its kept entries to its atom's
// lane-ordered row.  Positions come from LDS as in the pair passes when the
// block's window fits.
// With gather staging, a block whose window exceeds LDS (up to kGatherSpan
// slots) first marks the neighbours it keeps in a bitmap over its window,
// then lists the marked slots in ascending order (glist, gcnt) when there
// are at most as many as its stage holds, and writes each kept entry as 16 times its
// neighbour's rank in that list (the rank is the number of marked slots
// before it).  Otherwise gcnt is 0 and entries are slot offsets.
template <bool GATHER>
__global__ void __launch_bounds__(kBlock) k_prune(Dev S) {
  __shared__ int32_t ring_lds[16 * kBlock];
  __shared__ int4 lq[kStage + 1];
  __shared__ int32_t key[kBlock];
  // gather staging: the bitmap of kept neighbours over the window and the
  // marked slots before each of its words, in lq (not staged then)
  constexpr int kWords = kGatherSpan / 32;
  static_assert(2 * kWords * sizeof(uint32_t) <= sizeof(lq), "bitmap fits");
  uint32_t *bits = reinterpret_cast<uint32_t *>(lq);
  int32_t *wbase = reinterpret_cast<int32_t *>(bits + kWords);
  // and the kept entries of each lane's row chunks (8 bits per chunk, chunk
  // c of thread t at c * kBlock + t), for rows of at most kMaskChunks chunks
  constexpr int kMaskChunks = 32;
  static_assert(2 * kWords * sizeof(uint32_t) + kMaskChunks * kBlock <= sizeof(lq),
                "kept masks fit");
  uint8_t *kmask = reinterpret_cast<uint8_t *>(wbase + kWords);
  const WorkLists W = work_lists(S);
  const int nbl = W.count[1];
  const int32_t *blocks = W.blocks;
  for (int it = blockIdx.x; it < nbl; it += gridDim.x) {  // uniform
    const int blk = blocks[it];
    const int2 bm = S.bmap[blk];
    PairBlock B;
    B.blk = blk;
    B.t0 = bm.x;
    B.nt = bm.y;
    B.b0 = (int64_t)bm.x * kTile;
    B.p = threadIdx.x;
    B.valid = B.p < bm.y * kTile;
    B.i = B.b0 + B.p;
    B.n = 0;
    const bool rebuilt = rebuilds(S, S.tile_rep[B.t0]);  // uniform
    const int cap = block_stage(S, blk);  // stage of the block's class
    int lo, size;
    block_window(S, B, lo, size);
    const bool staged =
        size > 0 && size <= cap && stage(S, lq, B, lo, size, cap);
    // gather staging of this block (uniform)
    const bool gmark = GATHER && size > cap && size <= kGatherSpan;
    const int nwords = gmark ? (size + 31) >> 5 : 0;
    const int64_t i = B.b0 + B.p;
    const int n = B.valid ? S.nn[i] : 0;
    int64_t row = B.b0 + (B.valid ? (int)S.atom_lane[i] : 0);
    if (rebuilt) {
      // lane order of the pair passes: the block's atoms by descending list
      // length, ties by slot
      key[B.p] = lane_key(B.valid ? n : -1, B.p);
      __syncthreads();
      if (B.valid) {
        const int rank = lane_rank(key, B.p, B.nt);
        row = B.b0 + rank;
        S.lane_atom[row] = (uint8_t)B.p;
        S.atom_lane[i] = (uint8_t)rank;
      }
    }
    const int4 qi = B.valid ? S.qpos[i] : make_int4(0, 0, 0, 0);
    const float rp2 = S.prune_r2q;
    const int nch = S.k_cap >> 3;
    const int base = size > 0 ? lo : 0;  // entries are offsets from base
    auto kept = [&](const int4 &q, bool in) {
      const float dx = (float)(q.x - qi.x);
      const float dy = (float)(q.y - qi.y);
      const float dz = (float)(q.z - qi.z);
      return in & (fmaf(dx, dx, fmaf(dy, dy, dz * dz)) < rp2);
    };
    int gc = 0;  // listed neighbours when the block is gather-staged
    // the marking pass also records which entries it keeps, so that the
    // pass writing the rows needs no positions (uniform)
    const bool masked = gmark && S.k_cap <= 8 * kMaskChunks;
    if (gmark) {
      for (int w = threadIdx.x; w < nwords; w += kBlock) bits[w] = 0u;
      __syncthreads();
      chunk_loop(S.nl, S.N, i, (int)i, n, 0, 1, [&](const int (&j)[8], int k0) {
        int4 q[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) q[e] = gather_q(S.qpos, j[e]);
        uint32_t m = 0;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (kept(q[e], k0 + e < n)) {
            const uint32_t off = (uint32_t)(j[e] - lo);
            atomicOr(&bits[off >> 5], 1u << (off & 31));
            m |= 1u << e;
          }
        if (masked) kmask[(k0 >> 3) * kBlock + threadIdx.x] = (uint8_t)m;
      });
      __syncthreads();
      // each thread takes kWpt consecutive words
      constexpr int kWpt = kWords / kBlock;
      const int w0 = threadIdx.x * kWpt;
      int cnt = 0;
#pragma unroll
      for (int k = 0; k < kWpt; ++k)
        cnt += w0 + k < nwords ? __popc(bits[w0 + k]) : 0;
      int total = 0;
      int at = block_excl_scan(cnt, key, &total);
      if (total <= cap) {
        uint16_t *g = S.glist + (int64_t)blk * kStage;
#pragma unroll
        for (int k = 0; k < kWpt; ++k) {
          if (w0 + k < nwords) {
            wbase[w0 + k] = at;
            uint32_t m = bits[w0 + k];
            while (m) {
              const int b = __ffs(m) - 1;
              m &= m - 1u;
              g[at++] = (uint16_t)((w0 + k) * 32 + b);
            }
          }
        }
        gc = total;
      }
      __syncthreads();  // wbase complete
      if (threadIdx.x == 0) S.gcnt[blk] = gc;
    } else if (GATHER && threadIdx.x == 0) {
      S.gcnt[blk] = 0;
    }
    // entry of kept neighbour j: its rank in the gather list, or its offset
    auto entry = [&](int j) {
      if (gc > 0) {
        const uint32_t off = (uint32_t)(j - lo);
        const uint32_t w = off >> 5;
        return (int32_t)((uint32_t)(wbase[w] +
                                    __popc(bits[w] & ((1u << (off & 31)) - 1u)))
                         << 4);
      }
      return list_entry(j, base);
    };
    Ring ring{ring_lds + threadIdx.x, 0, 0};
    if (staged) {
      // the row in batches of kPruneBatch chunks, all loaded before any is
      // used: the stores of the ring's flushes then overlap the positions'
      // LDS reads instead of delaying the next list loads (loads and stores
      // retire in order)
      constexpr int kPruneBatch = GATHER ? 4 : 7;
      const StagedIndex sx(lo, cap);
      const int own = (n + 7) >> 3;
      const int4 *pad = reinterpret_cast<const int4 *>(kPadChunk);
      // the core: a row's leading ncore entries, within the core radius at
      // the build, stay in its pruned row until the next build.  After the
      // build's own pruning, a row's chunks that hold core entries only are
      // left as written (the block's window, and so the entries' encoding,
      // is fixed between builds): each lane starts at its first chunk past
      // them, and the other core entries are kept without a test.
      const int nc = S.core_r2q > 0.0f && B.valid ? S.ncore[i] : 0;
      const int cs = rebuilt ? 0 : nc >> 3;
      const int span = __builtin_amdgcn_readfirstlane(wave_max_i(own - cs));
      ring.cnt = ring.head = 8 * cs;
      for (int t0 = 0; t0 < span; t0 += kPruneBatch) {
        const int c0 = cs + t0;
        int4 buf[2 * kPruneBatch];
#pragma unroll
        for (int k = 0; k < kPruneBatch; ++k) {
          const int4 *src =
              c0 + k < own
                  ? reinterpret_cast<const int4 *>(S.nl + cl8(S.N, i, c0 + k))
                  : pad;
          buf[2 * k] = src[0];
          buf[2 * k + 1] = src[1];
        }
#pragma unroll
        for (int k = 0; k < kPruneBatch; ++k) {
          const int j[8] = {buf[2 * k].x,     buf[2 * k].y,     buf[2 * k].z,
                            buf[2 * k].w,     buf[2 * k + 1].x, buf[2 * k + 1].y,
                            buf[2 * k + 1].z, buf[2 * k + 1].w};
          int4 q[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) q[e] = sx.get(lq, j[e]);
          // pad entries read the sentinel, which lies beyond the pruning
          // radius, so they need no test of their own
          const int k0 = 8 * (c0 + k);
#pragma unroll
          for (int e = 0; e < 8; ++e)
            ring.put(list_entry(j[e], base), (k0 + e < nc) | kept(q[e], true));
          ring.flush(S.nl_lane, S.N, row, nch);
        }
      }
    } else if (masked) {
      // each thread reads back only the masks it wrote
      chunk_loop(S.nl, S.N, i, (int)i, n, 0, 1, [&](const int (&j)[8], int k0) {
        const uint32_t m = kmask[(k0 >> 3) * kBlock + threadIdx.x];
#pragma unroll
        for (int e = 0; e < 8; ++e) ring.put(entry(j[e]), ((m >> e) & 1u) != 0u);
        ring.flush(S.nl_lane, S.N, row, nch);
      });
    } else {
      chunk_loop(S.nl, S.N, i, (int)i, n, 0, 1, [&](const int (&j)[8], int k0) {
        int4 q[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) q[e] = gather_q(S.qpos, j[e]);
#pragma unroll
        for (int e = 0; e < 8; ++e) ring.put(entry(j[e]), kept(q[e], k0 + e < n));
        ring.flush(S.nl_lane, S.N, row, nch);
      });
    }
    if (B.valid) {
      ring.finish(S.nl_lane, S.N, row, nch,
                  gc > 0 ? pad_staged(cap) : pad_of_window(size, cap));
      S.nn_lane[row] = ring.cnt;
      // beside the pruning position, the atom's displacement since the list
      // build (quanta, one added for rounding): the position update bounds
      // the displacement since the build by its own since the pruning plus
      // this, without reading the build positions
      const double bx = S.x[i] - S.xr[i], by = S.y[i] - S.yr[i],
                   bz = S.z[i] - S.zr[i];
      const float db =
          (float)(sqrt(bx * bx + by * by + bz * bz) * S.qscale) + 1.0f;
      S.qprune[i] = make_int4(qi.x, qi.y, qi.z, __float_as_int(db));
    }
    __syncthreads();  // lq, bits, wbase and key serve the next block
  }
}

// One lane per atom: rho_i over the Verlet list, g_i = 1/sqrt(rho_i) into
// qpos[i].w.  With COUNT, nact[2i] and nact[2i+1] count the pairs with
// 0 < r <= r_tail and r_tail < r < r_cut.  Staged: positions from LDS, the
// unused entries hit the sentinel.  Not staged: global gathers, the unused
// entries are replaced by the atom itself and masked (r = 0); with GATHER
// the entries are ranks in the block's gather list (size = its length).
template <bool STAGED, bool COUNT, int STAGE, bool GATHER = false>
__device__ __forceinline__ void density_run(const Dev &S, const PotF &P,
                                            const PairBlock &B,
                                            const int4 *lq, int lo, int size) {
  const int64_t i = B.i;
  const bool valid = B.valid;
  const int self = valid ? (int)i : 0;
  const int4 qi = valid ? S.qpos[i] : make_int4(0, 0, 0, 0);
  const int n = B.n;
  const int64_t row = B.b0 + B.p;
  const int64_t N = S.N;
  const int4 *__restrict__ qp = S.qpos;
  const float aF = in_vgpr(P.aF), bF = in_vgpr(P.bF);
  const float uS = in_vgpr(P.uS), uB = in_vgpr(P.uB);
  const float fa = in_vgpr(P.fa), fb = in_vgpr(P.fb);
  const float rc2 = P.rc2, rt = P.rt;
  float rho = 0.0f;
  int nc = 0, nt = 0;
  auto pair = [&](const int4 &q) {
    const float dx = (float)(q.x - qi.x);
    const float dy = (float)(q.y - qi.y);
    const float dz = (float)(q.z - qi.z);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float rr = __builtin_amdgcn_sqrtf(r2);
    const float fc = __builtin_amdgcn_exp2f(fmaf(aF, rr, bF));
    const float u = fmaxf(fmaf(rr, uS, uB), 0.0f);
    const float ft = u * (u * fmaf(fb, u, fa));
    const bool tail = rr > rt;
    float f = tail ? ft : fc;
    if (!STAGED) f = r2 > 0.0f ? f : 0.0f;
    rho += f;
    if (COUNT) {
      const bool in = r2 < rc2 && r2 > 0.0f;
      nc += (in && !tail) ? 1 : 0;
      nt += (in && tail) ? 1 : 0;
    }
  };
  if (STAGED) {
    chunk_loop_padded(S.nl_lane, N, row, n, pad_chunk_staged<STAGE>(),
                      [&](const int (&e)[8]) {
                        int4 q[8];
#pragma unroll
                        for (int k = 0; k < 8; ++k) q[k] = lds_at(lq, e[k]);
#pragma unroll
                        for (int k = 0; k < 8; ++k) pair(q[k]);
                      });
  } else {
    auto unstaged = [&](const auto &dec) {
      chunk_loop(S.nl_lane, N, row, kPadWide, n, 0, 1,
                 [&](const int (&e)[8], int) {
                   int4 q[8];
#pragma unroll
                   for (int k = 0; k < 8; ++k) q[k] = gather_q(qp, dec(e[k]));
#pragma unroll
                   for (int k = 0; k < 8; ++k) pair(q[k]);
                 });
    };
    if (GATHER)
      unstaged(GatherDecode(S, B, lo, size, self));
    else
      unstaged(ListDecode(lo, size, self));
  }
  if (valid) {
    const float g = rho > 0.0f ? __builtin_amdgcn_rsqf(rho) : 0.0f;
    S.qpos[i].w = __float_as_int(g);
    if (COUNT) reinterpret_cast<int2 *>(S.nact)[i] = make_int2(nc, nt);
  }
}

// One launch per stage class: blocks base .. base + gridDim.x - 1 of the
// block map, all of stage STAGE.
template <bool COUNT, bool GATHER, int STAGE>
__global__ void __launch_bounds__(kBlock) k_density_mixed(Dev S, PotF P,
                                                          int base) {
  __shared__ int4 lq[STAGE + 1];
  const PairBlock B = pair_block(S, base);
  if (retired(S, S.tile_rep[B.t0])) return;  // uniform over the block
  int lo, size;
  block_window(S, B, lo, size);
  const int gc = GATHER && size > STAGE ? S.gcnt[B.blk] : 0;  // uniform
  if (size > 0 && size <= STAGE && stage(S, lq, B, lo, size, STAGE))
    density_run<true, COUNT, STAGE>(S, P, B, lq, lo, size);
  else if (gc > 0 && stage_gather(S, lq, B, lo, gc, STAGE))
    density_run<true, COUNT, STAGE>(S, P, B, lq, lo, gc);
  else if (gc > 0)
    density_run<false, COUNT, STAGE, true>(S, P, B, lq, lo, gc);
  else
    density_run<false, COUNT, STAGE>(S, P, B, lq, lo, size);
}

__device__ __forceinline__ double radial_d(const PotD &P, bool dens,
                                           double r) {
  if (r > P.rc) return 0.0;
  if (r <= P.rt) {
    return dens ? P.xi2 * exp(-P.k2q * (r / P.r0 - 1.0))
                : P.A * exp(-P.kp * (r / P.r0 - 1.0));
  }
  double t = (r - P.rt) / P.w;
  return dens ? fma(fma(fma(P.f3, t, P.f2), t, P.f1), t, P.f0)
              : fma(fma(fma(P.v3, t, P.v2), t, P.v1), t, P.v0);
}

__device__ __forceinline__ double dradial_d(const PotD &P, bool dens,
                                            double r) {
  if (r > P.rc) return 0.0;
  if (r <= P.rt) {
    return dens ? -(P.k2q / P.r0) * P.xi2 * exp(-P.k2q * (r / P.r0 - 1.0))
                : -(P.kp / P.r0) * P.A * exp(-P.kp * (r / P.r0 - 1.0));
  }
  double t = (r - P.rt) / P.w;
  return dens ? fma(fma(3.0 * P.f3, t, 2.0 * P.f2), t, P.f1) / P.w
              : fma(fma(3.0 * P.v3, t, 2.0 * P.v2), t, P.v1) / P.w;
}

__device__ __forceinline__ int32_t nl_entry(const Dev &S, int64_t i, int k) {
  return S.nl[cl8(S.N, i, k >> 3) + (k & 7)];
}

__global__ void __launch_bounds__(kBlock) k_density_fp64(Dev S, PotD P,
                                                         double *g) {
  int64_t b0 = xcd_block() * kBlock;
  int64_t i = b0 + threadIdx.x;
  bool valid = i < S.N;
  if (valid && retired(S, S.tile_rep[i / kTile])) return;  // whole wavefront
  int n = valid ? S.nn[i] : 0;
  double xi = valid ? S.x[i] : 0.0, yi = valid ? S.y[i] : 0.0,
         zi = valid ? S.z[i] : 0.0;
  double rho = 0.0;
  for (int k = 0; k < n; ++k) {
    int j = nl_entry(S, i, k);
    double dx = S.x[j] - xi, dy = S.y[j] - yi, dz = S.z[j] - zi;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (r > 0.0) rho += radial_d(P, true, r);
  }
  if (valid) g[i] = rho > 0.0 ? 1.0 / sqrt(rho) : 0.0;
}

// ---------------------------------------------------------------------------
// pass 2: forces, per-atom energies, per-tile sums of E and of the zz virial
// ---------------------------------------------------------------------------
// One lane per atom over its Verlet list (positions staged in LDS as in
// pass 1; q.w carries g_j).  Per pair (core r <= r_tail: exponentials of
// eqs 1-2; tail: the cubic tails, zero from r_cut on):
// E'_ij = 2V'(r) - (g_i+g_j) phi'(r)/2, F_i += E'_ij d/r, and with ENERGY
// also E_i += V(r), w_i += E'_ij dz^2 / (2r).  Without ENERGY (steps whose
// observables are not logged) e_atom and the tile sums are left unchanged.
//
// With KICK (the mixed step loops) the pass also ends the step for its atoms:
// the second half kick v += dt/2 F/m of the dynamic atoms, their kinetic
// partial sums and, on logged steps, the axial bins of the rupture gap.
// These are the same operations, in the same order and precision, as
// k_integrate_b, so the results do not depend on which of the two ran.
template <bool STAGED, bool ENERGY, bool KICK, int STAGE, bool GATHER = false>
__device__ __forceinline__ void force_run(const Dev &S, const PotF &P,
                                          const DevMD &M, const PairBlock &B,
                                          const int4 *lq, int lo, int size,
                                          double *lsum,
                                          float *fx, float *fy, float *fz,
                                          float *eat) {
  const int tid = threadIdx.x;
  const int64_t i = B.i;
  const bool valid = B.valid;
  const int self = valid ? (int)i : 0;
  const int4 qi = valid ? S.qpos[i] : make_int4(0, 0, 0, 0);
  const int n = B.n;
  const int64_t row = B.b0 + B.p;
  const float gi = __int_as_float(qi.w);
  const float hgi = 0.5f * gi;
  const int64_t N = S.N;
  const int4 *__restrict__ qp = S.qpos;
  const float aV = in_vgpr(P.aV), bW = in_vgpr(P.bW);
  const float aP = in_vgpr(P.aP), bP = in_vgpr(P.bP);
  const float uS = in_vgpr(P.uS), uB = in_vgpr(P.uB);
  const float d0 = in_vgpr(P.dv0), d1 = in_vgpr(P.dv1);
  const float p0 = in_vgpr(P.dp0), p1 = in_vgpr(P.dp1);
  const float va = P.va, vb = P.vb, bV = P.bV;
  const float rt = P.rt;
  float ax = 0.f, ay = 0.f, az = 0.f, ev = 0.f, wz = 0.f;
  auto pair = [&](const int4 &q) {
    const float dx = (float)(q.x - qi.x);
    const float dy = (float)(q.y - qi.y);
    const float dz = (float)(q.z - qi.z);
    const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    const float ri = __builtin_amdgcn_rsqf(r2);
    const float rr = r2 * ri;
    const float G = fmaf(0.5f, __int_as_float(q.w), hgi);
    // core: E' = (g_i+g_j)/2 (2q/r0) phi - (2p/r0) V
    const float eW = __builtin_amdgcn_exp2f(fmaf(aV, rr, bW));
    const float eP = __builtin_amdgcn_exp2f(fmaf(aP, rr, bP));
    const float epc = fmaf(G, eP, -eW);
    const float u = fmaxf(fmaf(rr, uS, uB), 0.0f);
    const float ept = u * fmaf(G, fmaf(p1, u, p0), fmaf(d1, u, d0));
    const bool tail = rr > rt;
    const bool on = STAGED || r2 > 0.0f;
    const float s = on ? (tail ? ept : epc) * ri : 0.0f;
    ax = fmaf(s, dx, ax);
    ay = fmaf(s, dy, ay);
    if (ENERGY) {
      const float Vt = u * (u * fmaf(vb, u, va));
      const float V = tail ? Vt : __builtin_amdgcn_exp2f(fmaf(aV, rr, bV));
      ev += on ? V : 0.0f;
      // f_z as the same fused multiply-add as without energies, so that the
      // forces, and the trajectory, do not depend on which steps are logged
      az = fmaf(s, dz, az);
      wz = fmaf(s * dz, dz, wz);
    } else {
      az = fmaf(s, dz, az);
    }
  };
  if (STAGED) {
    chunk_loop_padded(S.nl_lane, N, row, n, pad_chunk_staged<STAGE>(),
                      [&](const int (&e)[8]) {
                        // half a chunk of positions at a time (1 % faster
                        // steps than all eight at once)
                        int4 q[4];
#pragma unroll
                        for (int k = 0; k < 4; ++k) q[k] = lds_at(lq, e[k]);
#pragma unroll
                        for (int k = 0; k < 4; ++k) pair(q[k]);
                        asm volatile("" ::: "memory");
#pragma unroll
                        for (int k = 0; k < 4; ++k) q[k] = lds_at(lq, e[k + 4]);
#pragma unroll
                        for (int k = 0; k < 4; ++k) pair(q[k]);
                      });
  } else {
    auto unstaged = [&](const auto &dec) {
      chunk_loop(S.nl_lane, N, row, kPadWide, n, 0, 1,
                 [&](const int (&e)[8], int) {
                   int4 q[8];
#pragma unroll
                   for (int k = 0; k < 8; ++k) q[k] = gather_q(qp, dec(e[k]));
#pragma unroll
                   for (int k = 0; k < 8; ++k) pair(q[k]);
                 });
    };
    if (GATHER)
      unstaged(GatherDecode(S, B, lo, size, self));
    else
      unstaged(ListDecode(lo, size, self));
  }
  if (valid) {
    fx[i] = ax;
    fy[i] = ay;
    fz[i] = az;
  }
  double k2 = 0.0, kz = 0.0, gq = 0.0;
  const bool baro = KICK && M.baro_mass > 0.0;
  // the kinetic tile sums are read every step by the Nose-Hoover thermostat
  // and the barostat, otherwise only on logged steps (uniform)
  const int64_t sf = KICK ? S.callb[2] : 0;  // flags of this step
  const bool ksums =
      KICK && (M.nh_tau > 0.0 || baro || (sf & kStepLog) != 0);
  // the second half kick, unless the next step's first kernel does it
  // (DevMD::defer; uniform)
  const bool kick = KICK && (sf & kStepKick) != 0;
  if (kick && valid) {
    const int r = S.tile_rep[B.t0];
    const int64_t step = *M.step;
    const uint8_t f = S.flag[i];
    if (baro) gq = f == 2 ? (double)az : f == 1 ? -(double)az : 0.0;
    if (f != 3) {
      const double z = S.z[i];
      if (f == 0) {
        const double ac = 0.5 * M.dt * kAccel / S.mass;
        const double vx = fma(ac, (double)ax, S.vx[i]);
        const double vy = fma(ac, (double)ay, S.vy[i]);
        const double vz = fma(ac, (double)az, S.vz[i]);
        S.vx[i] = vx;
        S.vy[i] = vy;
        S.vz[i] = vz;
        const double wv = vz - stream_u(M, r, z, grip_top(M, r, step + 1));
        k2 = S.mass * (vx * vx + vy * vy + wv * wv);
        kz = S.mass * wv * wv;
      }
      if (sf & kStepLog) {
        // axial bins of width cell/2 for the rupture gap
        const int nb = 2 * S.grid_dim[3 * r + 2];
        const double t = floor((z - S.grid_lo[3 * r + 2]) * 2.0 * S.inv_cell);
        const int b = t >= 0.0 ? (t < (double)nb ? (int)t : nb - 1) : 0;
        const unsigned long long kk = dkey(z);
        atomicMin(&S.zbmin[(int64_t)r * S.max_zbins + b], kk);
        atomicMax(&S.zbmax[(int64_t)r * S.max_zbins + b], kk);
      }
    }
  }
  float e = 0.0f;
  if (ENERGY && valid) {
    e = ev - (gi > 0.0f ? 1.0f / gi : 0.0f);
    eat[i] = e;
  }
  if (ENERGY || ksums) {
    // per-tile sums in slot order: each atom's values go to LDS at its slot
    // in the block, then wavefront w sums tile t0 + w.  lsum shares its LDS
    // with the staged positions, which every wavefront must have finished
    // reading first.
    __syncthreads();
    if (valid) {
      if (ENERGY) {
        lsum[i - B.b0] = (double)e;
        lsum[kBlock + (i - B.b0)] = (double)wz * (double)P.wscale;
      }
      if (ksums) {
        lsum[2 * kBlock + (i - B.b0)] = k2;
        lsum[3 * kBlock + (i - B.b0)] = kz;
      }
      if (baro) lsum[4 * kBlock + (i - B.b0)] = gq;
    }
    __syncthreads();
    const int w = tid / kTile;
    if (w < B.nt) {
      double *pt = S.part + (int64_t)(B.t0 + w) * kNPart;
      if (ENERGY) {
        const double e_i = wave_sum(lsum[tid]);
        const double w_i = wave_sum(lsum[kBlock + tid]);
        if ((tid & 63) == 0) {
          pt[kPartE] = e_i;
          pt[kPartW] = w_i;
        }
      }
      if (ksums) {
        const double k_i = wave_sum(lsum[2 * kBlock + tid]);
        const double kz_i = wave_sum(lsum[3 * kBlock + tid]);
        if ((tid & 63) == 0) {
          pt[kPartK] = k_i;
          pt[kPartKz] = kz_i;
        }
      }
      if (baro) {
        const double q_i = wave_sum(lsum[4 * kBlock + tid]);
        if ((tid & 63) == 0) pt[kPartQ] = q_i;
      }
    }
  }
}

// One launch per stage class, as the density pass.
template <bool KICK, bool GATHER, int STAGE>
__global__ void __launch_bounds__(kBlock) k_force_mixed(Dev S, PotF P,
                                                        DevMD M, float *fx,
                                                        float *fy, float *fz,
                                                        float *eat, int base) {
  __shared__ int4 lq[STAGE + 1];
  // per-tile sums after the pair loop, in the staged positions' LDS
  static_assert(5 * kBlock * sizeof(double) <= sizeof(lq), "lsum fits");
  double *lsum = reinterpret_cast<double *>(lq);
  const PairBlock B = pair_block(S, base);
  if (retired(S, S.tile_rep[B.t0])) return;  // uniform over the block
  const bool energy =
      S.energies > 0 || (S.energies < 0 && (S.callb[2] & kStepLog) != 0);
  int lo, size;
  block_window(S, B, lo, size);
  const int gc = GATHER && size > STAGE ? S.gcnt[B.blk] : 0;  // uniform
  bool staged = false;
  if (size > 0 && size <= STAGE) {
    staged = stage(S, lq, B, lo, size, STAGE);
  } else if (gc > 0) {
    staged = stage_gather(S, lq, B, lo, gc, STAGE);
    size = gc;  // the staged (or decoded) list length from here on
  }
  if (staged) {
    if (energy)
      force_run<true, true, KICK, STAGE>(S, P, M, B, lq, lo, size, lsum, fx, fy,
                                         fz, eat);
    else
      force_run<true, false, KICK, STAGE>(S, P, M, B, lq, lo, size, lsum, fx,
                                          fy, fz, eat);
  } else if (gc > 0) {
    if (energy)
      force_run<false, true, KICK, STAGE, true>(S, P, M, B, lq, lo, size, lsum,
                                                fx, fy, fz, eat);
    else
      force_run<false, false, KICK, STAGE, true>(S, P, M, B, lq, lo, size,
                                                 lsum, fx, fy, fz, eat);
  } else {
    if (energy)
      force_run<false, true, KICK, STAGE>(S, P, M, B, lq, lo, size, lsum, fx,
                                          fy, fz, eat);
    else
      force_run<false, false, KICK, STAGE>(S, P, M, B, lq, lo, size, lsum, fx,
                                           fy, fz, eat);
  }
}

__global__ void __launch_bounds__(kBlock) k_force_fp64(Dev S, PotD P,
                                                       const double *g,
                                                       double *fx, double *fy,
                                                       double *fz,
                                                       double *eat) {
  int64_t b0 = xcd_block() * kBlock;
  int64_t i = b0 + threadIdx.x;
  bool valid = i < S.N;
  if (valid && retired(S, S.tile_rep[i / kTile])) return;  // whole wavefront
  int n = valid ? S.nn[i] : 0;
  double xi = valid ? S.x[i] : 0.0, yi = valid ? S.y[i] : 0.0,
         zi = valid ? S.z[i] : 0.0;
  double gi = valid ? g[i] : 0.0;
  double ax = 0, ay = 0, az = 0, ev = 0, wz = 0, rho = 0;
  for (int k = 0; k < n; ++k) {
    int j = nl_entry(S, i, k);
    double dx = S.x[j] - xi, dy = S.y[j] - yi, dz = S.z[j] - zi;
    double r = sqrt(dx * dx + dy * dy + dz * dz);
    if (!(r > 0.0) || r > P.rc) continue;
    double ep = 2.0 * dradial_d(P, false, r) -
                0.5 * (gi + g[j]) * dradial_d(P, true, r);
    double s = ep / r;
    ax += s * dx;
    ay += s * dy;
    az += s * dz;
    wz += s * dz * dz;
    ev += radial_d(P, false, r);
    rho += radial_d(P, true, r);
  }
  double e_i = 0.0, w_i = 0.0;
  if (valid) {
    double e = ev - sqrt(rho);
    fx[i] = ax;
    fy[i] = ay;
    fz[i] = az;
    eat[i] = e;
    e_i = e;
    w_i = 0.5 * wz;
  }
  e_i = wave_sum(e_i);
  w_i = wave_sum(w_i);
  if ((threadIdx.x & 63) == 0 && valid) {
    double *pt = S.part + (i / kTile) * kNPart;
    pt[kPartE] = e_i;
    pt[kPartW] = w_i;
  }
}

// ---------------------------------------------------------------------------
// integrator (BAOAB + grips) and per-replica reductions
// ---------------------------------------------------------------------------

template <typename FT, bool MIXED>
__global__ void __launch_bounds__(kBlock) k_integrate_a(Dev S, DevMD M,
                                                        const FT *fx,
                                                        const FT *fy,
                                                        const FT *fz) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool valid = i < S.N;
  int r = valid ? S.tile_rep[i / kTile] : 0;
  if (valid && (M.status[r] & 32u)) return;  // retired (whole wavefront)
  int64_t step = *M.step;
  const double dt = M.dt, hdt = 0.5 * dt;
  uint8_t f = valid ? S.flag[i] : 3;
  double disp2 = 0.0;
  float pd2 = 0.0f;  // |q - qprune|^2 (quanta^2) when pruning
  float dbq = 0.0f;  // displacement since the build at the last pruning
  // the previous step left its second half kick to this one (DevMD::defer):
  // it was neither logged nor the last of a call (uniform)
  const bool pend = MIXED && (S.callb[2] & kStepPend) != 0;
  if (f != 3) {
    double x = S.x[i], y = S.y[i], z = S.z[i];
    double vx = S.vx[i], vy = S.vy[i], vz = S.vz[i];
    if (f == 0) {
      const double ac = hdt * kAccel / S.mass;
      const double gx = (double)fx[i], gy = (double)fy[i], gz = (double)fz[i];
      // the kicks are explicit fused multiply-adds, the same as the force
      // pass's, so that a deferred kick rounds exactly as an immediate one
      if (pend) {
        vx = fma(ac, gx, vx);
        vy = fma(ac, gy, vy);
        vz = fma(ac, gz, vz);
      }
      if (M.nh_tau > 0.0) {
        // the thermostat half steps that end the last step and begin this
        // one, as one scale of the peculiar velocity
        const double sc = S.nhw[5 * r + kNhPend];
        const double u0 = stream_u(M, r, z, grip_top(M, r, step));
        vx *= sc;
        vy *= sc;
        vz = u0 + sc * (vz - u0);
      }
      vx = fma(ac, gx, vx);
      vy = fma(ac, gy, vy);
      vz = fma(ac, gz, vz);
      x += hdt * vx;
      y += hdt * vy;
      z += hdt * vz;
      if (M.gamma > 0.0) {
        double n0, n1, n2;
        uint32_t tag = atom_tag(S, r, i);
        if (MIXED) {  // FP32 Box-Muller on the same Philox words
          float m0, m1, m2;
          gauss3f(M.seed[r], (uint32_t)S.rep_id[r], tag, (uint64_t)step, 0u,
                  m0, m1, m2);
          n0 = m0;
          n1 = m1;
          n2 = m2;
        } else {
          gauss3(M.seed[r], (uint32_t)S.rep_id[r], tag, (uint64_t)step, 0u,
                 n0, n1, n2);
        }
        double sg = sqrt(kBoltz * target_T(M, r, (double)step + 0.5) /
                         S.mass * kAccel) *
                    sqrt(1.0 - M.c1 * M.c1);
        double uz = stream_u(M, r, z, M.v_pull[r] * ((double)step + 0.5) * dt);
        vx = M.c1 * vx + sg * n0;
        vy = M.c1 * vy + sg * n1;
        vz = uz + M.c1 * (vz - uz) + sg * n2;
      }
      x += hdt * vx;
      y += hdt * vy;
      z += hdt * vz;
      S.x[i] = x;
      S.y[i] = y;
      S.z[i] = z;
      S.vx[i] = vx;
      S.vy[i] = vy;
      S.vz[i] = vz;
    } else if (f == 1) {
      z = S.z0[i] - (M.baro_mass > 0.0 ? S.baw[2 * r + kBaS]
                                       : grip_bottom(M, step + 1));
      S.z[i] = z;
      S.vx[i] = 0.0;
      S.vy[i] = 0.0;
      S.vz[i] = 0.0;
    } else {
      const bool free = M.baro_mass > 0.0;
      z = S.z0[i] + (free ? S.baw[2 * r + kBaS] : grip_top(M, r, step + 1));
      S.z[i] = z;
      S.vx[i] = 0.0;
      S.vy[i] = 0.0;
      S.vz[i] = (M.grip_hold > 0 || free) ? 0.0 : M.v_pull[r];
    }
    if (MIXED) {
      bool out = false;
      const int4 q = quantise(S, r, i, x, y, z, out);
      if (out) atomicOr(&S.wstatus[r], 4u);
      if (S.pruning) {
        const int4 p = S.qprune[i];
        const float ex = (float)(q.x - p.x), ey = (float)(q.y - p.y),
                    ez = (float)(q.z - p.z);
        pd2 = fmaf(ex, ex, fmaf(ey, ey, ez * ez));
        if (out) pd2 = 3.0e38f;  // also NaN positions
        dbq = __int_as_float(p.w);
      }
    }
    if (!(MIXED && S.rebuild_bound)) {
      double ex = x - S.xr[i], ey = y - S.yr[i], ez = z - S.zr[i];
      disp2 = ex * ex + ey * ey + ez * ez;
      if (!(disp2 == disp2)) disp2 = 1.0e300;  // NaN forces a rebuild
    }
  }
  // per-replica flags (a NaN displacement counts as far).  With the pruning
  // bound, the displacement since the list build is at most the one since
  // the last pruning (from the quantised positions, plus two quanta for their
  // rounding) plus the one since the build at that pruning.
  const bool far = MIXED && S.rebuild_bound
                       ? !(sqrtf(pd2) + 2.0f + dbq <= S.skin_half_q)
                       : !(disp2 <= S.skin_half2);
  const bool pfar = MIXED && S.pruning && !(pd2 <= S.prune_d2q);
  const uint32_t m = (wave_any(far) ? 1u : 0u) | (wave_any(pfar) ? 2u : 0u);
  if ((threadIdx.x & 63) == 0 && valid && m) atomicOr(&S.rflag[r], m);
}

template <typename FT>
__global__ void __launch_bounds__(kBlock) k_integrate_b(Dev S, DevMD M,
                                                        const FT *fx,
                                                        const FT *fy,
                                                        const FT *fz) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool valid = i < S.N;
  int r = valid ? S.tile_rep[i / kTile] : 0;
  if (valid && (M.status[r] & 32u)) return;  // retired (whole wavefront)
  int64_t step = *M.step;
  const double hdt = 0.5 * M.dt;
  uint8_t f = valid ? S.flag[i] : 3;
  double k2 = 0.0, kz = 0.0;
  const bool logstep = (S.callb[2] & kStepLog) != 0;
  const bool baro = M.baro_mass > 0.0;
  const double gq = !baro ? 0.0
                    : f == 2 ? (double)fz[i]
                    : f == 1 ? -(double)fz[i]
                             : 0.0;
  if (f != 3) {
    double z = S.z[i];
    if (f == 0) {
      double ac = hdt * kAccel / S.mass;
      double vx = S.vx[i] + ac * (double)fx[i];
      double vy = S.vy[i] + ac * (double)fy[i];
      double vz = S.vz[i] + ac * (double)fz[i];
      S.vx[i] = vx;
      S.vy[i] = vy;
      S.vz[i] = vz;
      double wv = vz - stream_u(M, r, z, grip_top(M, r, step + 1));
      k2 = S.mass * (vx * vx + vy * vy + wv * wv);
      kz = S.mass * wv * wv;
    }
    if (logstep) {
      // axial bins of width cell/2 for the rupture gap
      int nb = 2 * S.grid_dim[3 * r + 2];
      double t = floor((z - S.grid_lo[3 * r + 2]) * 2.0 * S.inv_cell);
      int b = t >= 0.0 ? (t < (double)nb ? (int)t : nb - 1) : 0;
      unsigned long long kk = dkey(z);
      atomicMin(&S.zbmin[(int64_t)r * S.max_zbins + b], kk);
      atomicMax(&S.zbmax[(int64_t)r * S.max_zbins + b], kk);
    }
  }
  k2 = wave_sum(k2);
  kz = wave_sum(kz);
  const double q = baro ? wave_sum(gq) : 0.0;
  if ((threadIdx.x & 63) == 0 && valid) {
    double *pt = S.part + (i / kTile) * kNPart;
    pt[kPartK] = k2;
    pt[kPartKz] = kz;
    if (baro) pt[kPartQ] = q;
  }
}

// Deterministic block sum of the partials of tiles [t0, t1) (entries k0..k1).
template <int NV>
__device__ __forceinline__ void block_sum_tiles(const double *part,
                                                int64_t t0, int64_t t1,
                                                int k0, double *out,
                                                double *lds /* [NV*256] */) {
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int64_t t = t0 + threadIdx.x; t < t1; t += blockDim.x) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += part[t * kNPart + k0 + v];
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) lds[v * 256 + threadIdx.x] = acc[v];
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
        lds[v * 256 + threadIdx.x] += lds[v * 256 + threadIdx.x + s];
    }
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = lds[v * 256];
}

__global__ void __launch_bounds__(256) k_reduce_forces(Dev S, double *rep_e,
                                                       double *rep_w) {
  __shared__ double lds[2 * 256];
  int r = blockIdx.x;
  int64_t t0 = S.rep_off[r] / kTile, t1 = S.rep_off[r + 1] / kTile;
  double s[2];
  block_sum_tiles<2>(S.part, t0, t1, kPartE, s, lds);
  if (threadIdx.x == 0) {
    rep_e[r] = s[0];
    rep_w[r] = s[1];
  }
}

// End of a step, one workgroup per replica: sums, observables, status.  The
// step index and the next step's flags are advanced by k_step_advance, the
// next kernel on the stream.  (A last-workgroup ticket would save that launch
// but costs a device-wide fence in every workgroup, which is dearer.)
__global__ void __launch_bounds__(256) k_reduce_step(Dev S, DevMD M) {
  __shared__ double lds[5 * 256];
  int r = blockIdx.x;
  int64_t step = *M.step;
  int64_t n1 = step + 1;
  int64_t t0 = S.rep_off[r] / kTile, t1 = S.rep_off[r + 1] / kTile;
  // energy and virial tile sums are current on logged steps only
  const bool logstep = (S.callb[2] & kStepLog) != 0;  // n1 % n_log == 0
  const bool frozen = (M.status[r] & 32u) != 0;  // retired: record unchanged
  // (each sum is the same whichever other entries are summed with it)
  const bool baro = M.baro_mass > 0.0;
  // the kinetic sums are current every step only when the thermostat or the
  // barostat reads them (they then also serve the finiteness check);
  // otherwise they are summed on logged steps, which also check finiteness
  double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (logstep) {
    if (baro)
      block_sum_tiles<5>(S.part, t0, t1, kPartE, s, lds);
    else
      block_sum_tiles<4>(S.part, t0, t1, kPartE, s, lds);
  } else if (baro) {
    block_sum_tiles<3>(S.part, t0, t1, kPartK, s + 2, lds);
  } else if (M.nh_tau > 0.0) {
    block_sum_tiles<2>(S.part, t0, t1, kPartK, s + 2, lds);
  }
  int nb = 2 * S.grid_dim[3 * r + 2];
  unsigned long long *bmin = S.zbmin + (int64_t)r * S.max_zbins;
  unsigned long long *bmax = S.zbmax + (int64_t)r * S.max_zbins;
  if (threadIdx.x == 0 && !frozen) {
    double E = s[0], wzz = s[1];
    double KE = 0.5 * s[2] / kAccel, Kz = s[3] / kAccel;
    if (M.nh_tau > 0.0) {
      // thermostat half step that ends this step (its scale is applied by
      // the next step's first kick, or when the call ends), then the one
      // that begins the next step
      double *w = S.nhw + 5 * r;
      double zeta = w[kNhZeta], eta = w[kNhEta];
      const double Tn = target_T(M, r, (double)n1);
      const double sb = nh_half(M, r, Tn, zeta, eta, KE);
      Kz *= sb * sb;
      M.nh_xi[r] = zeta;
      if (M.nh_eta) M.nh_eta[r] = eta;
      double K2 = KE;
      const double sa = nh_half(M, r, Tn, zeta, eta, K2);
      w[kNhPend] = sb * sa;
      w[kNhEnd] = sb;
      w[kNhZeta] = zeta;
      w[kNhEta] = eta;
      w[kNhTop] = grip_top(M, r, n1);
    }
    int dof = M.dof[r];
    double T = dof > 0 ? 2.0 * KE / ((double)dof * kBoltz) : 0.0;
    double D = elongation(M, r, n1);
    if (baro) {
      // barostat: second half kick of ds/dt with the grip force of the new
      // positions, then the first half kick and the drift of the next step
      double *bw = S.baw + 2 * r;
      const double Q = s[4];
      const double damp = exp(-0.5 * M.baro_damp * M.dt);
      const double sn = bw[kBaS];
      const double vn = baro_kick(M, bw[kBaV], Q) * damp;
      M.baro_s[2 * r] = sn;
      M.baro_s[2 * r + 1] = vn;
      const double vh = baro_kick(M, vn * damp, Q);
      bw[kBaV] = vh;
      bw[kBaS] = sn + M.dt * vh;
      D = 2.0 * sn;
    }
    uint32_t st = S.wstatus[r];
    if (!isfinite(E) || !isfinite(KE)) st |= 2u;  // E is 0 when not logged
    if (S.rflag[r] & 1u) st |= 16u;
    if (logstep) {
      double gap = 0.0, pmax = 0.0;
      bool have = false;
      for (int b = 0; b < nb; ++b) {
        unsigned long long mn = bmin[b];
        if (mn == ~0ull) continue;
        if (have) gap = fmax(gap, dkey_inv(mn) - pmax);
        pmax = dkey_inv(bmax[b]);
        have = true;
      }
      if (gap >= M.r_cut) st |= 8u;
      // retirement: `retire` A of grip travel after the first rupture
      if (M.retire > 0.0) {
        if ((st & 8u) && M.dfail[r] < 0.0) M.dfail[r] = D;
        if (M.dfail[r] >= 0.0 && D >= M.dfail[r] + M.retire) st |= 32u;
      }
      double *o = M.obs + ((n1 / M.n_log) % M.n_slots) * (int64_t)S.R * 10 +
                  (int64_t)r * 10;
      o[0] = (double)n1;
      o[1] = E;
      o[2] = KE;
      o[3] = T;
      o[4] = wzz;
      o[5] = (wzz - Kz) / M.vol[r] * kEvA3ToGPa;
      o[6] = D / M.L0[r];
      o[7] = gap;
      o[8] = D;
      o[9] = (double)(M.status[r] | st);
    }
    M.status[r] |= st;
    S.wstatus[r] = 0u;
    S.rflag[r] = 0u;
  } else if (threadIdx.x == 0 && logstep) {
    // a retired replica repeats its last record (with its step index)
    const int64_t k = n1 / M.n_log;
    const double *src = M.obs + ((k - 1) % M.n_slots) * (int64_t)S.R * 10 +
                        (int64_t)r * 10;
    double *dst = M.obs + (k % M.n_slots) * (int64_t)S.R * 10 + (int64_t)r * 10;
    if (k > 0)
      for (int q = 0; q < 10; ++q) dst[q] = src[q];
  }
  __syncthreads();
  if (logstep) {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) {
      bmin[b] = ~0ull;
      bmax[b] = 0ull;
    }
  }
}

// The step index and the flags of the step it now names.
__global__ void k_step_advance(DevMD M, int64_t *callb) {
  const int64_t n1 = *M.step + 1;
  *M.step = n1;
  callb[2] = step_flags(M, callb, n1);
}

// ---------------------------------------------------------------------------
// Nose-Hoover thermostat: the first half step of a call's first step, and
// the last end-of-step scale applied when the call ends.  Inside a call the
// two half steps between consecutive steps are folded into kNhPend.
// ---------------------------------------------------------------------------
// The start of a step-loop call: the first Nose-Hoover half step, from the
// kinetic energy of the velocities as they are; the barostat's first half
// kick and drift, from the grip force of the forces in `out` (summed per tile
// and per replica exactly as the step loops sum it).
template <typename FT>
__global__ void __launch_bounds__(256) k_step_begin(Dev S, DevMD M,
                                                    const FT *fz) {
  __shared__ double lds[256];
  const int r = blockIdx.x;
  const bool gone = (M.status[r] & 32u) != 0;  // retired (uniform per block)
  const int64_t step = *M.step;
  if (M.nh_tau > 0.0) {
    double *w = S.nhw + 5 * r;
    if (gone) {  // nothing pending
      if (threadIdx.x == 0) {
        w[kNhPend] = 1.0;
        w[kNhEnd] = 1.0;
      }
    } else {
      const double top = grip_top(M, r, step);
      double k2 = 0.0;
      for (int64_t i = S.rep_off[r] + threadIdx.x; i < S.rep_off[r + 1];
           i += blockDim.x) {
        if (S.flag[i] != 0) continue;
        const double vx = S.vx[i], vy = S.vy[i];
        const double wz = S.vz[i] - stream_u(M, r, S.z[i], top);
        k2 += S.mass * (vx * vx + vy * vy + wz * wz);
      }
      lds[threadIdx.x] = k2;
      __syncthreads();
      for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) lds[threadIdx.x] += lds[threadIdx.x + o];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        double K = 0.5 * lds[0] / kAccel;
        double zeta = M.nh_xi[r], eta = M.nh_eta ? M.nh_eta[r] : 0.0;
        w[kNhPend] =
            nh_half(M, r, target_T(M, r, (double)step), zeta, eta, K);
        w[kNhEnd] = 1.0;
        w[kNhZeta] = zeta;
        w[kNhEta] = eta;
        w[kNhTop] = top;
      }
      __syncthreads();
    }
  }
  if (M.baro_mass > 0.0 && !gone) {
    const int64_t t0 = S.rep_off[r] / kTile, t1 = S.rep_off[r + 1] / kTile;
    const int lane = threadIdx.x & 63;
    for (int64_t t = t0 + (threadIdx.x >> 6); t < t1; t += blockDim.x >> 6) {
      const int64_t i = t * kTile + lane;
      const uint8_t f = S.flag[i];
      const double g = f == 2   ? (double)fz[i]
                       : f == 1 ? -(double)fz[i]
                                : 0.0;
      const double q = wave_sum(g);
      if (lane == 0) S.part[t * kNPart + kPartQ] = q;
    }
    __threadfence_block();
    __syncthreads();
    double Q;
    block_sum_tiles<1>(S.part, t0, t1, kPartQ, &Q, lds);
    if (threadIdx.x == 0) {
      double *bw = S.baw + 2 * r;
      const double damp = exp(-0.5 * M.baro_damp * M.dt);
      const double vh = baro_kick(M, M.baro_s[2 * r + 1] * damp, Q);
      bw[kBaV] = vh;
      bw[kBaS] = M.baro_s[2 * r] + M.dt * vh;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_nh_finish(Dev S, DevMD M) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= S.N || S.flag[i] != 0) return;
  const int r = S.tile_rep[i / kTile];
  const double *w = S.nhw + 5 * r;
  const double sb = w[kNhEnd];
  if (sb == 1.0) return;
  const double u = stream_u(M, r, S.z[i], w[kNhTop]);
  S.vx[i] *= sb;
  S.vy[i] *= sb;
  S.vz[i] = u + sb * (S.vz[i] - u);
}

// ---------------------------------------------------------------------------
// initial state
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) k_init_a(Dev S, DevMD M,
                                                   double jitter) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool valid = i < S.N;
  int r = valid ? S.tile_rep[i / kTile] : 0;
  uint8_t f = valid ? S.flag[i] : 3;
  double sx = 0, sy = 0, sz = 0, cn = 0;
  if (f != 3) {
    uint32_t tag = atom_tag(S, r, i);
    uint32_t rid = (uint32_t)S.rep_id[r];
    if (jitter != 0.0) {
      uint4 o = rng_words(M.seed[r], rid, tag, 0, 2u);
      S.x[i] += jitter * (2.0 * u01(o.x) - 1.0);
      S.y[i] += jitter * (2.0 * u01(o.y) - 1.0);
      S.z[i] += jitter * (2.0 * u01(o.z) - 1.0);
    }
    double vx = 0, vy = 0, vz = 0;
    if (f == 0) {
      double sg = sqrt(kBoltz * target_T(M, r, 0.0) / S.mass * kAccel);
      double n0, n1, n2;
      gauss3(M.seed[r], rid, tag, 0, 1u, n0, n1, n2);
      vx = sg * n0;
      vy = sg * n1;
      vz = sg * n2;
      sx = vx;
      sy = vy;
      sz = vz;
      cn = 1.0;
    } else if (f == 2 && M.grip_hold == 0 && M.baro_mass <= 0.0) {
      vz = M.v_pull[r];  // pulled grip (it rests under the barostat)
    }
    S.vx[i] = vx;
    S.vy[i] = vy;
    S.vz[i] = vz;
  }
  sx = wave_sum(sx);
  sy = wave_sum(sy);
  sz = wave_sum(sz);
  cn = wave_sum(cn);
  if ((threadIdx.x & 63) == 0 && valid) {
    double *pt = S.part + (i / kTile) * kNPart;
    pt[kPartA + 0] = sx;
    pt[kPartA + 1] = sy;
    pt[kPartA + 2] = sz;
    pt[kPartA + 3] = cn;
  }
}

// mode 0: centre-of-mass velocity -> rsum[8r..8r+2]; mode 1: rescale factor
// -> rsum[8r+3].
__global__ void __launch_bounds__(256) k_init_reduce(Dev S, DevMD M,
                                                     int mode) {
  __shared__ double lds[4 * 256];
  int r = blockIdx.x;
  int64_t t0 = S.rep_off[r] / kTile, t1 = S.rep_off[r + 1] / kTile;
  double s[4];
  block_sum_tiles<4>(S.part, t0, t1, kPartA, s, lds);
  if (threadIdx.x == 0) {
    double *rs = S.rsum + 8 * r;
    if (mode == 0) {
      double c = s[3] > 0.0 ? s[3] : 1.0;
      rs[0] = s[0] / c;
      rs[1] = s[1] / c;
      rs[2] = s[2] / c;
    } else {
      int dof = M.dof[r];
      double s2 = s[0];
      rs[3] = (s2 > 0.0 && dof > 0)
                  ? sqrt((double)dof * kBoltz * target_T(M, r, 0.0) /
                         (S.mass * s2 / kAccel))
                  : 0.0;
    }
  }
}

__global__ void __launch_bounds__(kBlock) k_init_b(Dev S) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  bool valid = i < S.N;
  int r = valid ? S.tile_rep[i / kTile] : 0;
  uint8_t f = valid ? S.flag[i] : 3;
  double s2 = 0.0;
  if (f == 0) {
    const double *rs = S.rsum + 8 * r;
    double vx = S.vx[i] - rs[0], vy = S.vy[i] - rs[1], vz = S.vz[i] - rs[2];
    S.vx[i] = vx;
    S.vy[i] = vy;
    S.vz[i] = vz;
    s2 = vx * vx + vy * vy + vz * vz;
  }
  s2 = wave_sum(s2);
  if ((threadIdx.x & 63) == 0 && valid) {
    double *pt = S.part + (i / kTile) * kNPart;
    pt[kPartA + 0] = s2;
    pt[kPartA + 1] = 0.0;
    pt[kPartA + 2] = 0.0;
    pt[kPartA + 3] = 0.0;
  }
}

template <bool MIXED>
__global__ void __launch_bounds__(kBlock) k_init_c(Dev S, DevMD M) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= S.N) return;
  int r = S.tile_rep[i / kTile];
  uint8_t f = S.flag[i];
  if (f == 3) {
    if (MIXED) S.qpos[i] = make_int4(0, 0, 0, 0);
    return;
  }
  double z = S.z[i];
  if (f == 0) {
    double sc = S.rsum[8 * r + 3];
    S.vx[i] *= sc;
    S.vy[i] *= sc;
    S.vz[i] = S.vz[i] * sc + stream_u(M, r, z, 0.0);
  }
  S.z0[i] = z;
  if (MIXED) {
    bool out = false;
    quantise(S, r, i, S.x[i], S.y[i], z, out);
    if (out) atomicOr(&S.wstatus[r], 4u);
  }
}

// Per-replica constants from the atoms as they are (one workgroup per
// replica): dof = 3 N_dyn - 3 (0 when N_dyn <= 1); vol = N (4/3) pi r_hs^3
// with r_hs = r0/2 and N the replica's atoms (eq 5's constant volume);
// z_lo / z_hi the inner faces of the fixed and pulled grips (largest z of
// the fixed grip, smallest z of the pulled one; the replica's lowest and
// highest z when it has no such grip).  Counts, minima and maxima are
// exact, so the result does not depend on the reduction order.
__global__ void __launch_bounds__(256) k_replica_constants(Dev S, double r0,
                                                           int32_t *dof,
                                                           double *vol,
                                                           double *z_lo,
                                                           double *z_hi) {
  __shared__ double red[4][4];
  __shared__ int cnt[4][2];
  const int r = blockIdx.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int ndyn = 0, nreal = 0;
  double gmax = -INFINITY, pmin = INFINITY, zmin = INFINITY, zmax = -INFINITY;
  for (int64_t i = S.rep_off[r] + threadIdx.x; i < S.rep_off[r + 1]; i += 256) {
    const uint8_t f = S.flag[i];
    if (f == 3) continue;
    const double z = S.z[i];
    ++nreal;
    ndyn += f == 0 ? 1 : 0;
    if (f == 1) gmax = gmax > z ? gmax : z;
    if (f == 2) pmin = pmin < z ? pmin : z;
    zmin = zmin < z ? zmin : z;
    zmax = zmax > z ? zmax : z;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ndyn += __shfl_xor(ndyn, o, 64);
    nreal += __shfl_xor(nreal, o, 64);
    gmax = fmax(gmax, __shfl_xor(gmax, o, 64));
    pmin = fmin(pmin, __shfl_xor(pmin, o, 64));
    zmin = fmin(zmin, __shfl_xor(zmin, o, 64));
    zmax = fmax(zmax, __shfl_xor(zmax, o, 64));
  }
  if (lane == 0) {
    cnt[w][0] = ndyn;
    cnt[w][1] = nreal;
    red[w][0] = gmax;
    red[w][1] = pmin;
    red[w][2] = zmin;
    red[w][3] = zmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      ndyn += cnt[k][0];
      nreal += cnt[k][1];
      gmax = fmax(gmax, red[k][0]);
      pmin = fmin(pmin, red[k][1]);
      zmin = fmin(zmin, red[k][2]);
      zmax = fmax(zmax, red[k][3]);
    }
    dof[r] = ndyn > 1 ? 3 * ndyn - 3 : 0;
    const double rhs = 0.5 * r0;
    vol[r] = (double)nreal * (4.0 / 3.0) * 3.14159265358979323846 * (rhs * rhs * rhs);
    z_lo[r] = gmax > -INFINITY ? gmax : zmin;
    z_hi[r] = pmin < INFINITY ? pmin : zmax;
  }
}

// The current state as the start of a new stretch (step loops' observables):
// grip references z0 = z for every atom; each replica's initial length L0
// grows by the barostat's elongation 2 s, whose s and ds/dt are zeroed.
__global__ void __launch_bounds__(kBlock) k_rebase(Dev S, double *L0,
                                                   double *baro_s) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < S.N) S.z0[i] = S.z[i];
  if (i < S.R) {
    if (baro_s != nullptr) {
      L0[i] += 2.0 * baro_s[2 * i];
      baro_s[2 * i] = 0.0;
      baro_s[2 * i + 1] = 0.0;
    }
  }
}

__global__ void k_rng_fill(uint64_t seed, uint32_t rep, uint64_t step,
                           uint32_t stream, int64_t n, uint32_t *w,
                           double *g, float *gf) {
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  if (w) {
    uint4 o = rng_words(seed, rep, (uint32_t)t, step, stream);
    w[4 * t + 0] = o.x;
    w[4 * t + 1] = o.y;
    w[4 * t + 2] = o.z;
    w[4 * t + 3] = o.w;
  }
  if (g) {
    double a, b, c;
    gauss3(seed, rep, (uint32_t)t, step, stream, a, b, c);
    g[3 * t + 0] = a;
    g[3 * t + 1] = b;
    g[3 * t + 2] = c;
  }
  if (gf) {
    float a, b, c;
    gauss3f(seed, rep, (uint32_t)t, step, stream, a, b, c);
    gf[3 * t + 0] = a;
    gf[3 * t + 1] = b;
    gf[3 * t + 2] = c;
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b) {
  return (unsigned)((n + b - 1) / b);
}

void launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v,
                     hipStream_t s) {
  if (n > 0) k_fill_u64<<<nblk(n, 256), 256, 0, s>>>(p, n, v);
}
void launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
  if (n > 0) k_fill_u32<<<nblk(n, 256), 256, 0, s>>>(p, n, v);
}
void launch_set_step(int64_t *p, int64_t v, hipStream_t s) {
  k_set_step<<<1, 1, 0, s>>>(p, v);
}
void launch_quantise(const Dev &S, hipStream_t s) {
  k_quantise<<<nblk(S.N, kBlock), kBlock, 0, s>>>(S);
}

// Grid of the kernels that loop over a work list.
constexpr int64_t kWorkGrid = 2048;

static inline unsigned work_grid(int64_t items) {
  return (unsigned)std::max<int64_t>(1, std::min(items, kWorkGrid));
}

void launch_worklist(const Dev &S, hipStream_t s) {
  if (S.R > 0) k_worklist<<<1, 1024, 0, s>>>(S);
}

void launch_cells(const Dev &S, hipStream_t s) {
  if (S.R == 0) return;
  const int64_t nt = S.N / kTile;
  k_cell_count<<<work_grid((nt + 3) / 4), kBlock, 0, s>>>(S);
  k_cell_scan<<<work_grid(std::min<int64_t>(S.R, 256)), 1024, 0, s>>>(S);
  k_cell_fill<<<work_grid((nt + 3) / 4), kBlock, 0, s>>>(S);
  if (S.ncbmap > 0) k_cell_sort<<<work_grid(S.ncbmap), kBlock, 0, s>>>(S);
}

void launch_nlist(const Dev &S, bool mixed, double rl, hipStream_t s) {
  const double rq = rl * S.qscale;
  if (S.nbmap == 0) return;
  if (mixed) {
    // the rows of the rebuilt replicas, then the lane-ordered rows of the
    // rebuilt and the pruned ones (work lists of the step)
    k_nlist_mixed<<<work_grid(S.N / kTile), kNlBlock, 0, s>>>(S,
                                                          (float)(rq * rq));
    if (S.gather)
      k_prune<true><<<work_grid(S.nbmap), kBlock, 0, s>>>(S);
    else
      k_prune<false><<<work_grid(S.nbmap), kBlock, 0, s>>>(S);
  } else {
    k_nlist_fp64<<<S.nbmap, kBlock, 0, s>>>(S, rl * rl);
  }
}

// Sums of the full and of the lane-ordered list lengths (diagnostics).
__global__ void __launch_bounds__(kBlock) k_list_stats(Dev S, int mixed) {
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  long long a = 0, b = 0;
  if (i < S.N) {
    a = S.nn[i];
    b = mixed ? S.nn_lane[i] : a;
  }
  __shared__ long long ls[2][kBlock / kTile];
  a = wave_sum_ll(a);
  b = wave_sum_ll(b);
  if ((threadIdx.x & 63) == 0) {
    ls[0][threadIdx.x / kTile] = a;
    ls[1][threadIdx.x / kTile] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long sa = 0, sb = 0;
    for (int w = 0; w < kBlock / kTile; ++w) {
      sa += ls[0][w];
      sb += ls[1][w];
    }
    atomicAdd(&S.stats[0], (unsigned long long)sa);
    atomicAdd(&S.stats[1], (unsigned long long)sb);
  }
}

// How the pair passes reach the neighbours of each block (mixed precision):
// stats[2] blocks whose slot window fits LDS, stats[3] blocks staged through
// their gather lists, stats[4] the others (global gathers), stats[5] the
// neighbours listed by the gather-staged blocks.
__global__ void __launch_bounds__(kBlock) k_stage_stats(Dev S) {
  const int64_t b = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (b >= S.nbmap) return;
  const int2 bm = S.bmap[b];
  int l = 0x7fffffff, h = 0;
  bool ok = true;
  for (int t = 0; t < bm.y; ++t) {
    const int2 w = S.win[bm.x + t];
    ok = ok && w.y > w.x;
    l = min(l, w.x);
    h = max(h, w.y);
  }
  const int size = ok ? h - l : 0;
  const int cap = block_stage(S, b);
  const int gc = size > cap && S.gather ? S.gcnt[b] : 0;
  if (size > 0 && size <= cap)
    atomicAdd(&S.stats[2], 1ull);
  else if (gc > 0) {
    atomicAdd(&S.stats[3], 1ull);
    atomicAdd(&S.stats[5], (unsigned long long)gc);
  } else
    atomicAdd(&S.stats[4], 1ull);
}

void launch_list_stats(const Dev &S, bool mixed, hipStream_t s) {
  k_fill_u64<<<1, 64, 0, s>>>(S.stats, 6, 0ull);
  k_list_stats<<<nblk(S.N, kBlock), kBlock, 0, s>>>(S, mixed ? 1 : 0);
  if (mixed && S.nbmap > 0)
    k_stage_stats<<<nblk(S.nbmap, kBlock), kBlock, 0, s>>>(S);
}

void launch_block_map(const Dev &S, hipStream_t s) {
  k_block_map<<<1, 1024, 0, s>>>(S);
  k_cell_map<<<1, 1024, 0, s>>>(S);
}

// The mixed pair passes: one launch per stage class that has blocks, each in
// its gather-staging variant when the system enables it (the other variant
// has none of its code).
template <bool GATHER, int C>
void density_class(const Dev &S, const PotF &PF, hipStream_t s) {
  constexpr int ST = stage_of_class(C);
  const int base = S.cls_off[C], nb = S.cls_off[C + 1] - base;
  if (nb <= 0) return;
  if (S.nact)
    k_density_mixed<true, GATHER, ST><<<nb, kBlock, 0, s>>>(S, PF, base);
  else
    k_density_mixed<false, GATHER, ST><<<nb, kBlock, 0, s>>>(S, PF, base);
}
template <bool GATHER>
void density_pass(const Dev &S, const PotF &PF, hipStream_t s) {
  density_class<GATHER, 0>(S, PF, s);
  density_class<GATHER, 1>(S, PF, s);
}
void density_pass(const Dev &S, const PotF &PF, hipStream_t s) {
  if (S.gather)
    density_pass<true>(S, PF, s);
  else
    density_pass<false>(S, PF, s);
}
template <bool KICK, bool GATHER, int C>
void force_class(const Dev &S, const PotF &PF, const DevMD &M, void *fx,
                 void *fy, void *fz, void *eat, hipStream_t s) {
  constexpr int ST = stage_of_class(C);
  const int base = S.cls_off[C], nb = S.cls_off[C + 1] - base;
  if (nb <= 0) return;
  k_force_mixed<KICK, GATHER, ST><<<nb, kBlock, 0, s>>>(
      S, PF, M, (float *)fx, (float *)fy, (float *)fz, (float *)eat, base);
}
template <bool KICK>
void force_pass(const Dev &S, const PotF &PF, const DevMD &M, void *fx,
                void *fy, void *fz, void *eat, hipStream_t s) {
  if (S.gather) {
    force_class<KICK, true, 0>(S, PF, M, fx, fy, fz, eat, s);
    force_class<KICK, true, 1>(S, PF, M, fx, fy, fz, eat, s);
  } else {
    force_class<KICK, false, 0>(S, PF, M, fx, fy, fz, eat, s);
    force_class<KICK, false, 1>(S, PF, M, fx, fy, fz, eat, s);
  }
}

void launch_forces(const Dev &S, bool mixed, const PotF &PF, const PotD &PD,
                   void *fx, void *fy, void *fz, void *eat, double *g,
                   hipStream_t s) {
  unsigned nb = nblk(S.N, kBlock);
  if (mixed) {
    if (S.nbmap == 0) return;
    density_pass(S, PF, s);
    force_pass<false>(S, PF, DevMD{}, fx, fy, fz, eat, s);
  } else {
    k_density_fp64<<<nb, kBlock, 0, s>>>(S, PD, g);
    k_force_fp64<<<nb, kBlock, 0, s>>>(S, PD, g, (double *)fx, (double *)fy,
                                       (double *)fz, (double *)eat);
  }
}

void launch_forces_kick(const Dev &S, const DevMD &M, const PotF &PF,
                        void *fx, void *fy, void *fz, void *eat,
                        hipStream_t s) {
  if (S.nbmap == 0) return;
  density_pass(S, PF, s);
  force_pass<true>(S, PF, M, fx, fy, fz, eat, s);
}

void launch_force_pass(const Dev &S, bool mixed, int pass, const PotF &PF,
                       const PotD &PD, void *fx, void *fy, void *fz, void *eat,
                       double *g, hipStream_t s) {
  unsigned nb = nblk(S.N, kBlock);
  if (mixed) {
    if (S.nbmap == 0) return;
    if (pass == 1)
      density_pass(S, PF, s);
    else
      force_pass<false>(S, PF, DevMD{}, fx, fy, fz, eat, s);
  } else {
    if (pass == 1)
      k_density_fp64<<<nb, kBlock, 0, s>>>(S, PD, g);
    else
      k_force_fp64<<<nb, kBlock, 0, s>>>(S, PD, g, (double *)fx, (double *)fy,
                                         (double *)fz, (double *)eat);
  }
}

void launch_reduce_forces(const Dev &S, double *re, double *rw,
                          hipStream_t s) {
  k_reduce_forces<<<S.R, 256, 0, s>>>(S, re, rw);
}

void launch_integrate_a(const Dev &S, const DevMD &M, bool mixed,
                        const void *fx, const void *fy, const void *fz,
                        hipStream_t s) {
  unsigned nb = nblk(S.N, kBlock);
  if (mixed)
    k_integrate_a<float, true><<<nb, kBlock, 0, s>>>(
        S, M, (const float *)fx, (const float *)fy, (const float *)fz);
  else
    k_integrate_a<double, false><<<nb, kBlock, 0, s>>>(
        S, M, (const double *)fx, (const double *)fy, (const double *)fz);
}

void launch_integrate_b(const Dev &S, const DevMD &M, bool mixed,
                        const void *fx, const void *fy, const void *fz,
                        hipStream_t s) {
  unsigned nb = nblk(S.N, kBlock);
  if (mixed)
    k_integrate_b<float><<<nb, kBlock, 0, s>>>(
        S, M, (const float *)fx, (const float *)fy, (const float *)fz);
  else
    k_integrate_b<double><<<nb, kBlock, 0, s>>>(
        S, M, (const double *)fx, (const double *)fy, (const double *)fz);
}

__global__ void k_call_bounds(DevMD M, int64_t *callb, int64_t n) {
  const int64_t m = *M.step;
  callb[0] = m;
  callb[1] = m + n;
  callb[2] = step_flags(M, callb, m);
}

void launch_call_bounds(const Dev &S, const DevMD &M, int64_t n,
                        hipStream_t s) {
  k_call_bounds<<<1, 1, 0, s>>>(M, S.callb, n);
}

void launch_reduce_step(const Dev &S, const DevMD &M, hipStream_t s) {
  k_reduce_step<<<S.R, 256, 0, s>>>(S, M);
  k_step_advance<<<1, 1, 0, s>>>(M, S.callb);
}

void launch_step_begin(const Dev &S, const DevMD &M, bool mixed,
                       const void *fz, hipStream_t s) {
  if (mixed)
    k_step_begin<float><<<S.R, 256, 0, s>>>(S, M, (const float *)fz);
  else
    k_step_begin<double><<<S.R, 256, 0, s>>>(S, M, (const double *)fz);
}

void launch_nh_finish(const Dev &S, const DevMD &M, hipStream_t s) {
  k_nh_finish<<<nblk(S.N, kBlock), kBlock, 0, s>>>(S, M);
}

void launch_init(const Dev &S, const DevMD &M, bool mixed, double jitter,
                 hipStream_t s) {
  unsigned nb = nblk(S.N, kBlock);
  k_init_a<<<nb, kBlock, 0, s>>>(S, M, jitter);
  k_init_reduce<<<S.R, 256, 0, s>>>(S, M, 0);
  k_init_b<<<nb, kBlock, 0, s>>>(S);
  k_init_reduce<<<S.R, 256, 0, s>>>(S, M, 1);
  if (mixed)
    k_init_c<true><<<nb, kBlock, 0, s>>>(S, M);
  else
    k_init_c<false><<<nb, kBlock, 0, s>>>(S, M);
}

void launch_rng_fill(uint64_t seed, uint32_t rep, uint64_t step,
                     uint32_t stream, int64_t n, uint32_t *w, double *g,
                     float *gf, hipStream_t s) {
  if (n > 0)
    k_rng_fill<<<nblk(n, 256), 256, 0, s>>>(seed, rep, step, stream, n, w, g,
                                            gf);
}

void launch_replica_constants(const Dev &S, double r0, int32_t *dof,
                              double *vol, double *z_lo, double *z_hi,
                              hipStream_t s) {
  if (S.R > 0)
    k_replica_constants<<<S.R, 256, 0, s>>>(S, r0, dof, vol, z_lo, z_hi);
}

void launch_rebase(const Dev &S, double *L0, double *baro_s, hipStream_t s) {
  const int64_t n = std::max<int64_t>(S.N, S.R);
  if (n > 0) k_rebase<<<nblk(n, kBlock), kBlock, 0, s>>>(S, L0, baro_s);
}

}  // namespace tbsma
