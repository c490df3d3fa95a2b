// RowSampling on the product distribution and the merge of duplicate samples
// (Definition of leverage score sampling; Algorithm 2 sampling lines; the
// diagonal view of S and the distinct prefix sets of Theorem
// kron_mat_mul_sqrt_decomp).
//
//   k_sample        Philox4x64-10 words -> per-mode inverse-CDF draws -> packed key
//   k_radix_*       stable LSD radix sort of the packed keys (8- or 9-bit digits)
//   k_tree_*        run-length encoding of the sorted keys at every prefix length:
//                   the nodes of level k are the distinct (i_0..i_{k-1})
//   k_rows          per distinct row: multiplicity, merged weight
//                   Omega_j = count_j / (m prod_n p'_{i_n}), gathered response b_j
//
// The packed key stores mode n's index in bits [shift[n], shift[n] + bits[n]),
// mode 0 most significant, so sorting keys sorts rows by their linear index and
// every prefix of modes is a contiguous key range.
#include "kr_internal.h"

namespace kr {

#define SORT_THREADS 256
#define SORT_ITEMS 16
#define SORT_TILE (SORT_THREADS * SORT_ITEMS)
// The tree kernels take smaller tiles than the sort: their work per key is a few
// compares, so a launch wants many workgroups rather than long per-thread runs.
#define TREE_ITEMS 4
#define TREE_TILE (SORT_THREADS * TREE_ITEMS)
#define SORT_DIGITS_MAX 512   // histogram rows per tile (9-bit digits at most)

// ---------------------------------------------------------------------------
// Sampling.  CDF tables are staged in LDS when they fit (cdf_in_lds != 0).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_sample(ModeTables T, Geom g, uint64_t seed, uint64_t stream,
                                                uint64_t row, int cdf_in_lds,
                                                uint64_t* __restrict__ keys) {
  extern __shared__ uint64_t lds_cdf[];
  const uint64_t* C[KR_MAXN];
  int off = 0;
  for (int n = 0; n < g.N; ++n) {
    if (cdf_in_lds) {
      for (int i = threadIdx.x; i < g.I[n]; i += blockDim.x) lds_cdf[off + i] = T.C[n][i];
      C[n] = lds_cdf + off;
    } else {
      C[n] = T.C[n];
    }
    off += g.I[n];
  }
  __syncthreads();
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < g.m;
       t += (int64_t)gridDim.x * blockDim.x) {
    uint64_t key = 0;
    // the caller's mode o draws from word o % 4 of block (t, o / 4, row, 0); it is
    // tree mode n = inv[o] (the same mode unless the modes were reordered)
    for (int grp = 0; grp * 4 < g.N; ++grp) {
      const u64x4 w = philox4x64_10((uint64_t)t, (uint64_t)grp, row, 0ull, seed, stream);
      for (int k = 0; k < 4 && grp * 4 + k < g.N; ++k) {
        const int n = g.inv[grp * 4 + k];
        const uint64_t u = w.v[k] >> 32;
        // number of CDF entries <= u  (index i with C_{i-1} <= u < C_i)
        int lo = 0, hi = g.I[n];
        const uint64_t* c = C[n];
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (c[mid] <= u) lo = mid + 1; else hi = mid;
        }
        key |= (uint64_t)lo << g.shift[n];
      }
    }
    keys[t] = key;
  }
}

// Every problem of a batch in one launch: job j owns blocks [b0_j, b0_{j+1}) and
// draws its m_j samples exactly as k_sample does (the key of sample t depends on t
// only, so the grid does not change any key).  Each block stages its problem's
// CDFs in LDS when they fit.
struct SampleJob {
  const uint64_t* C[KR_MAXN];
  int I[KR_MAXN];
  int shift[KR_MAXN];
  int inv[KR_MAXN];
  int N;
  int64_t m;
  uint64_t seed, stream;
  uint64_t* keys;
  int64_t b0;            // first block of the job
};

#define SB_LDS_ENTRIES 4096
__global__ void __launch_bounds__(256) k_sample_batched(const SampleJob* __restrict__ jobs, int njobs) {
  __shared__ uint64_t cdf[SB_LDS_ENTRIES];
  __shared__ int jsh;
  if (threadIdx.x == 0) {
    int lo = 0, hi = njobs - 1;   // last job with b0 <= blockIdx.x
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (jobs[mid].b0 <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    jsh = lo;
  }
  __syncthreads();
  const SampleJob& jb = jobs[jsh];
  const int64_t b1 = jsh + 1 < njobs ? jobs[jsh + 1].b0 : (int64_t)gridDim.x;
  const int N = jb.N;
  int sumI = 0;
  for (int n = 0; n < N; ++n) sumI += jb.I[n];
  const bool in_lds = sumI <= SB_LDS_ENTRIES;
  const uint64_t* C[KR_MAXN];
  int off = 0;
  for (int n = 0; n < N; ++n) {
    if (in_lds) {
      for (int i = threadIdx.x; i < jb.I[n]; i += blockDim.x) cdf[off + i] = jb.C[n][i];
      C[n] = cdf + off;
    } else {
      C[n] = jb.C[n];
    }
    off += jb.I[n];
  }
  __syncthreads();
  const int64_t nthr = (b1 - jb.b0) * (int64_t)blockDim.x;
  for (int64_t t = (blockIdx.x - jb.b0) * (int64_t)blockDim.x + threadIdx.x; t < jb.m; t += nthr) {
    uint64_t key = 0;
    for (int grp = 0; grp * 4 < N; ++grp) {
      const u64x4 w = philox4x64_10((uint64_t)t, (uint64_t)grp, 0ull, 0ull, jb.seed, jb.stream);
      for (int k = 0; k < 4 && grp * 4 + k < N; ++k) {
        const int n = jb.inv[grp * 4 + k];
        const uint64_t u = w.v[k] >> 32;
        int lo = 0, hi = jb.I[n];
        const uint64_t* c = C[n];
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (c[mid] <= u) lo = mid + 1; else hi = mid;
        }
        key |= (uint64_t)lo << jb.shift[n];
      }
    }
    jb.keys[t] = key;
  }
}

// ---------------------------------------------------------------------------
// LSD radix sort, RB-bit digits (8 or 9: 27-bit keys sort in three passes of 9
// bits instead of four of 8).  hist is digit-major: hist[d * nblocks + b], with
// room for SORT_DIGITS_MAX digits.
// ---------------------------------------------------------------------------
// BMAJ: the counts are stored tile-major (hist[tile NB + digit]) for the scatter
// that forms its own offsets; else digit-major, the order of the global scan.
template <int RB, bool BMAJ = false>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_hist(const uint64_t* __restrict__ keys, int64_t m,
                                                            int shift, uint32_t* __restrict__ hist,
                                                            int nblocks) {
  constexpr int NB = 1 << RB;
  static_assert(NB <= SORT_DIGITS_MAX && NB % SORT_THREADS == 0, "digit count");
  __shared__ uint32_t cnt[NB];
  for (int d = threadIdx.x; d < NB; d += SORT_THREADS) cnt[d] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
  for (int k = 0; k < SORT_ITEMS; ++k) {
    const int64_t t = base + (int64_t)k * SORT_THREADS + threadIdx.x;
    if (t < m) atomicAdd(&cnt[(keys[t] >> shift) & (uint64_t)(NB - 1)], 1u);
  }
  __syncthreads();
  for (int d = threadIdx.x; d < NB; d += SORT_THREADS)
    hist[BMAJ ? (size_t)blockIdx.x * NB + d : (size_t)d * nblocks + blockIdx.x] = cnt[d];
}

// Exclusive scan of n uint32 values in place, in tiles of NT SCAN_K entries:
// each thread loads its SCAN_K consecutive entries with 16-byte loads and scans
// them in registers, the thread totals are scanned inside each wave by shuffles
// and the NT / 64 wave totals are read by every thread (two workgroup barriers
// per tile).  scan_tile scans the tile at t0 on top of carry and returns the
// tile's total.
#define SCAN_K 48
template <int NT>
__device__ __forceinline__ uint32_t scan_tile(uint32_t* __restrict__ v, int64_t n, int64_t t0, uint32_t carry,
                                              uint32_t* wsum) {
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int64_t c0 = t0 + (int64_t)threadIdx.x * SCAN_K;
  const bool full = c0 + SCAN_K <= n;   // v is 16-byte aligned and c0 a multiple of 4
  uint32_t x[SCAN_K];
  if (full) {
#pragma unroll
    for (int q = 0; q < SCAN_K / 4; ++q) {
      const uint4 u = reinterpret_cast<const uint4*>(v + c0)[q];
      x[4 * q] = u.x;
      x[4 * q + 1] = u.y;
      x[4 * q + 2] = u.z;
      x[4 * q + 3] = u.w;
    }
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_K; ++j) x[j] = c0 + j < n ? v[c0 + j] : 0u;
  }
  uint32_t tot = 0u;
#pragma unroll
  for (int j = 0; j < SCAN_K; ++j) {
    const uint32_t t = x[j];
    x[j] = tot;
    tot += t;
  }
  uint32_t inc = tot;   // inclusive scan of the thread totals within the wave
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t up = __shfl_up(inc, o, 64);
    if (lane >= o) inc += up;
  }
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  uint32_t before = 0u, total = 0u;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    const uint32_t t = wsum[i];
    before += i < wv ? t : 0u;
    total += t;
  }
  const uint32_t base = carry + before + inc - tot;
  if (full) {
#pragma unroll
    for (int q = 0; q < SCAN_K / 4; ++q) {
      uint4 u;
      u.x = base + x[4 * q];
      u.y = base + x[4 * q + 1];
      u.z = base + x[4 * q + 2];
      u.w = base + x[4 * q + 3];
      reinterpret_cast<uint4*>(v + c0)[q] = u;
    }
  } else {
#pragma unroll
    for (int j = 0; j < SCAN_K; ++j)
      if (c0 + j < n) v[c0 + j] = base + x[j];
  }
  __syncthreads();   // wsum is rewritten by the next tile
  return total;
}

// One workgroup of 1024 threads over all tiles, a running carry linking them.
// The histogram scans of the sort at 340k keys (512 x 84 entries) take one tile.
__global__ void __launch_bounds__(1024) k_scan_u32(uint32_t* __restrict__ v, int64_t n) {
  __shared__ uint32_t wsum[16];
  uint32_t carry = 0u;
  for (int64_t t0 = 0; t0 < n; t0 += 1024 * SCAN_K) carry += scan_tile<1024>(v, n, t0, carry, wsum);
}

// Longer scans over many workgroups, one tile of SCANP_THREADS SCAN_K entries
// each: k_scan_part writes the tiles' totals, k_scan_tiles scans every tile on
// top of the sum of the totals before it (integer sums: the same result as one
// workgroup's running carry).
#define SCANP_THREADS 256
#define SCANP_TILE (SCANP_THREADS * SCAN_K)
__global__ void __launch_bounds__(SCANP_THREADS) k_scan_part(const uint32_t* __restrict__ v, int64_t n,
                                                            uint32_t* __restrict__ part) {
  __shared__ uint32_t wsum[SCANP_THREADS / 64];
  const int64_t c0 = (int64_t)blockIdx.x * SCANP_TILE + (int64_t)threadIdx.x * SCAN_K;
  uint32_t tot = 0u;
  if (c0 + SCAN_K <= n) {
#pragma unroll
    for (int q = 0; q < SCAN_K / 4; ++q) {
      const uint4 u = reinterpret_cast<const uint4*>(v + c0)[q];
      tot += u.x + u.y + u.z + u.w;
    }
  } else {
    for (int j = 0; j < SCAN_K; ++j) tot += c0 + j < n ? v[c0 + j] : 0u;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = tot;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0u;
    for (int i = 0; i < SCANP_THREADS / 64; ++i) t += wsum[i];
    part[blockIdx.x] = t;
  }
}
__global__ void __launch_bounds__(SCANP_THREADS) k_scan_tiles(uint32_t* __restrict__ v, int64_t n,
                                                             const uint32_t* __restrict__ part) {
  __shared__ uint32_t wsum[SCANP_THREADS / 64];
  __shared__ uint32_t carry_s;
  uint32_t c = 0u;
  for (int b = threadIdx.x; b < (int)blockIdx.x; b += SCANP_THREADS) c += part[b];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0u;
    for (int i = 0; i < SCANP_THREADS / 64; ++i) t += wsum[i];
    carry_s = t;
  }
  __syncthreads();
  const uint32_t carry = carry_s;
  __syncthreads();   // wsum is reused by the tile scan
  scan_tile<SCANP_THREADS>(v, n, (int64_t)blockIdx.x * SCANP_TILE, carry, wsum);
}

// Stable scatter.  The tile is processed in rounds of SORT_THREADS consecutive
// keys; in a round, a key's rank among equal digits is (earlier waves' counts) +
// (earlier lanes in its wave with the same digit, found by ballot matching over
// the RB + 1 bits of the digit, NB marking an absent key).
// OWN: hist holds the raw per-tile counts, tile-major, and every workgroup forms
// its own offsets (used for few tiles, where reading the whole histogram per
// workgroup costs less than a separate scan launch): thread t owns the digits
// d = t NB / SORT_THREADS + i, sums each digit's counts over all tiles and over
// the tiles before its own (one coalesced read of a tile's row per step), and an
// exclusive scan of the digit totals across the workgroup adds the digits before d.
template <int RB, bool OWN = false>
__global__ void __launch_bounds__(SORT_THREADS) k_radix_scatter(const uint64_t* __restrict__ in,
                                                               uint64_t* __restrict__ out, int64_t m,
                                                               int shift, const uint32_t* __restrict__ hist,
                                                               int nblocks) {
  constexpr int NB = 1 << RB;
  constexpr int NW = SORT_THREADS / 64;
  __shared__ uint32_t base_[NB];
  __shared__ uint32_t wcnt[NW][NB + 1];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if constexpr (OWN) {
    constexpr int DPT = NB / SORT_THREADS;   // digits per thread
    uint32_t tot[DPT], bef[DPT], sum = 0u;
#pragma unroll
    for (int i = 0; i < DPT; ++i) tot[i] = bef[i] = 0u;
    const uint32_t* __restrict__ col = hist + threadIdx.x * DPT;
#pragma unroll 4
    for (int k = 0; k < nblocks; ++k) {
      uint32_t c[DPT];
      if constexpr (DPT == 2) {
        const uint2 v = *reinterpret_cast<const uint2*>(col + (size_t)k * NB);
        c[0] = v.x;
        c[1] = v.y;
      } else {
#pragma unroll
        for (int i = 0; i < DPT; ++i) c[i] = col[(size_t)k * NB + i];
      }
#pragma unroll
      for (int i = 0; i < DPT; ++i) {
        tot[i] += c[i];
        bef[i] += k < (int)blockIdx.x ? c[i] : 0u;
      }
    }
#pragma unroll
    for (int i = 0; i < DPT; ++i) sum += tot[i];
    // exclusive scan of the threads' digit totals: within the wave, then the waves
    uint32_t inc = sum;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t up = __shfl_up(inc, o, 64);
      if (lane >= o) inc += up;
    }
    if (lane == 63) wcnt[w][0] = inc;
    __syncthreads();
    uint32_t run = inc - sum;
    for (int k = 0; k < w; ++k) run += wcnt[k][0];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < DPT; ++i) {
      base_[threadIdx.x * DPT + i] = run + bef[i];
      run += tot[i];
    }
    for (int d = threadIdx.x; d < NB; d += SORT_THREADS)
      for (int k = 0; k < NW; ++k) wcnt[k][d] = 0;
  } else {
    for (int d = threadIdx.x; d < NB; d += SORT_THREADS) {
      base_[d] = hist[(size_t)d * nblocks + blockIdx.x];
      for (int k = 0; k < NW; ++k) wcnt[k][d] = 0;
    }
  }
  if (threadIdx.x < NW) wcnt[threadIdx.x][NB] = 0;
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
  const int64_t tbase = (int64_t)blockIdx.x * SORT_TILE;
  for (int r = 0; r < SORT_ITEMS; ++r) {
    const int64_t t = tbase + (int64_t)r * SORT_THREADS + threadIdx.x;
    const bool valid = t < m;
    const uint64_t key = valid ? in[t] : 0ull;
    const uint32_t d = valid ? (uint32_t)((key >> shift) & (uint64_t)(NB - 1)) : (uint32_t)NB;
    unsigned long long peers = ~0ull;
#pragma unroll
    for (int b = 0; b <= RB; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = __popcll(peers & lt);
    if (rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = base_[d] + rank;
      for (int k = 0; k < w; ++k) pos += wcnt[k][d];
      out[pos] = key;
    }
    __syncthreads();
    for (int dd = threadIdx.x; dd < NB; dd += SORT_THREADS) {
      uint32_t add = 0;
      for (int k = 0; k < NW; ++k) { add += wcnt[k][dd]; wcnt[k][dd] = 0; }
      base_[dd] += add;
    }
    if (threadIdx.x < NW) wcnt[threadIdx.x][NB] = 0;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Tree build: flag_k[t] = (t == 0) or prefix_k(key[t]) != prefix_k(key[t-1]).
// Pass 1 counts flags per tile and level; pass 2 scans tile totals; pass 3
// assigns node ids and writes node arrays.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t level_flags(const uint64_t* keys, int64_t t, const Geom& g) {
  if (t == 0) return (1u << (g.N + 1)) - 2u;  // levels 1..N
  const uint64_t a = keys[t], b = keys[t - 1];
  uint32_t f = 0;
  for (int k = 1; k <= g.N; ++k)
    if ((a >> g.lshift[k]) != (b >> g.lshift[k])) f |= 1u << k;
  return f;
}

__global__ void __launch_bounds__(SORT_THREADS) k_tree_count(const uint64_t* __restrict__ keys, Geom g,
                                                            int64_t* __restrict__ tiletot) {
  __shared__ int64_t red[SORT_THREADS / 64][KR_MAXN + 1];
  int cnt[KR_MAXN + 1];
  for (int k = 0; k <= KR_MAXN; ++k) cnt[k] = 0;
  // items t = tile + e SORT_THREADS + thread: the key loads are coalesced
  const int64_t t0 = (int64_t)blockIdx.x * TREE_TILE + threadIdx.x;
  for (int e = 0; e < TREE_ITEMS; ++e) {
    const int64_t t = t0 + (int64_t)e * SORT_THREADS;
    if (t < g.m) {
      const uint32_t f = level_flags(keys, t, g);
      for (int k = 1; k <= g.N; ++k) cnt[k] += (f >> k) & 1u;
    }
  }
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int k = 1; k <= g.N; ++k) {
    int v = cnt[k];
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) red[w][k] = v;
  }
  __syncthreads();
  if (threadIdx.x <= (unsigned)g.N && threadIdx.x >= 1) {
    int64_t s = 0;
    for (int k = 0; k < SORT_THREADS / 64; ++k) s += red[k][threadIdx.x];
    tiletot[(size_t)blockIdx.x * (KR_MAXN + 1) + threadIdx.x] = s;
  }
}

// Exclusive scan over the tiles of each level's node counts: wave k - 1 scans
// level k (k = 1..N) 64 tiles at a time (a shuffle scan with a running carry),
// so the tiles' loads are issued 64 at a time instead of one after another.
// Launched with 64 N threads.
__global__ void k_tree_scan(int64_t* __restrict__ tiletot, int ntiles, Geom g, Tree tr) {
  const int lane = threadIdx.x & 63;
  const int k = (int)(threadIdx.x >> 6) + 1;
  if (threadIdx.x == 0) tr.cnt[0] = 1;
  if (k > g.N) return;
  int64_t run = 0;
  for (int b0 = 0; b0 < ntiles; b0 += 64) {
    const int b = b0 + lane;
    const int64_t v = b < ntiles ? tiletot[(size_t)b * (KR_MAXN + 1) + k] : 0;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t up = __shfl_up(inc, o, 64);
      if (lane >= o) inc += up;
    }
    if (b < ntiles) tiletot[(size_t)b * (KR_MAXN + 1) + k] = run + inc - v;
    run += __shfl(inc, 63, 64);
  }
  if (lane == 0) tr.cnt[k] = run;
}

__global__ void k_tree_sentinels(Geom g, Tree tr) {
  const int k = threadIdx.x;
  if (k < g.N) tr.fchild[k][tr.cnt[k]] = (int32_t)tr.cnt[k + 1];
  if (k == 0) {
    tr.fchild[0][0] = 0;
    tr.rstart[tr.cnt[g.N]] = (int32_t)g.m;
  }
}

// The tree's arrays from the sorted keys, one workgroup per tile.  The tile's
// items are taken in rounds of SORT_THREADS consecutive keys (coalesced loads):
// in a round, an item's rank among the round's level-k flags comes from a
// ballot, the waves' counts are exchanged through LDS, and per-level running
// counts carry the ranks across rounds; node s of level k is then written at
// tile offset + rank, with its parent (the level-(k-1) nodes started up to and
// including the item, less one) and its first child (the level-(k+1) nodes
// started before the item).
__global__ void __launch_bounds__(SORT_THREADS) k_tree_emit(const uint64_t* __restrict__ keys, Geom g,
                                                           const int64_t* __restrict__ tiletot, Tree tr) {
  constexpr int NW = SORT_THREADS / 64;
  __shared__ int wcnt[2][NW][KR_MAXN + 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;   // lanes below this one
  const int N = g.N;
  int64_t base[KR_MAXN + 2];   // level-k nodes before this round (tile offset included)
  for (int k = 0; k <= KR_MAXN + 1; ++k) base[k] = 0;
  for (int k = 1; k <= N; ++k) base[k] = tiletot[(size_t)blockIdx.x * (KR_MAXN + 1) + k];
  const int64_t tb = (int64_t)blockIdx.x * TREE_TILE;
  for (int e = 0; e < TREE_ITEMS; ++e) {
    const int64_t t = tb + (int64_t)e * SORT_THREADS + threadIdx.x;
    const bool in = t < g.m;
    const uint32_t f = in ? level_flags(keys, t, g) : 0u;
    const uint64_t key = in ? keys[t] : 0ull;
    const int buf = e & 1;
    int before[KR_MAXN + 2];   // level-k flags of earlier items in this round
    for (int k = 1; k <= N; ++k) {
      const uint64_t m = __ballot((f >> k) & 1u);
      before[k] = __popcll(m & lt);
      if (lane == 0) wcnt[buf][w][k] = __popcll(m);
    }
    __syncthreads();
    int64_t excl[KR_MAXN + 2];
    excl[0] = 0;
    excl[N + 1] = 0;
    for (int k = 1; k <= N; ++k) {
      int wb = 0, tot = 0;
      for (int q = 0; q < NW; ++q) {
        const int c = wcnt[buf][q][k];
        wb += q < w ? c : 0;
        tot += c;
      }
      excl[k] = base[k] + wb + before[k];
      base[k] += tot;
    }
    if (in) {
      for (int k = 1; k <= N; ++k) {
        if ((f >> k) & 1u) {
          const int64_t sk = excl[k];
          const int n = k - 1;
          tr.idx[k][sk] = (int32_t)((key >> g.shift[n]) & ((1ull << g.bits[n]) - 1ull));
          tr.parent[k][sk] = k == 1 ? 0 : (int32_t)(excl[k - 1] + ((f >> (k - 1)) & 1u) - 1);
          if (k < N) tr.fchild[k][sk] = (int32_t)excl[k + 1];
          if (k == N) {
            tr.rstart[sk] = (int32_t)t;
            tr.rkey[sk] = key;
          }
        }
      }
    }
    // wcnt[buf] is read again only two rounds later, after the next barrier
  }
}

// Gather the factor row of every tree node of levels up to kmax:
// arow[k][s][r] = A_{k-1}[idx[k][s]][r].
__global__ void __launch_bounds__(256) k_node_rows(ModeTables T, Geom g, Tree tr, int kmax) {
  for (int k = g.seg_root ? 2 : 1; k <= kmax; ++k) {
    const int R = g.R[k - 1];
    const int64_t total = tr.cnt[k] * R;
    const double* __restrict__ A = T.A[k - 1];
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
      const int64_t s = e / R;
      tr.arow[k][e] = A[(int64_t)tr.idx[k][s] * R + (e - s * R)];
    }
  }
}

// ---------------------------------------------------------------------------
// Distinct rows: multiplicity, Omega_j = count_j * omega_j with
// omega_j = 1 / (m prod_n Q_n[i_n] 2^-32) multiplied in mode order, gathered b.
// b is row-major (prod I) x nrhs of dtype b_dtype; bD is D x nrhs float64.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_rows(ModeTables T, Geom g, Tree tr, const void* __restrict__ b,
                                             int b_dtype, double* __restrict__ Omega,
                                             double* __restrict__ bD, int32_t* __restrict__ counts,
                                             int32_t* __restrict__ flags) {
  const int64_t D = tr.cnt[g.N];
  int bad = 0;
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < D;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = tr.rstart[j + 1] - tr.rstart[j];
    const uint64_t key = tr.rkey[j];
    double den = (double)g.m;
    int64_t lin = 0;
    for (int o = 0; o < g.N; ++o) {   // in the caller's mode order
      const int n = g.inv[o];
      const int i = (int)((key >> g.shift[n]) & ((1ull << g.bits[n]) - 1ull));
      den = den * ((double)T.Q[n][i] * 0x1p-32);
      lin = lin * g.I[n] + i;
    }
    const double om = 1.0 / den;
    Omega[j] = (double)c * om;
    counts[j] = c;
    if (!b) continue;   // implicit response: k_gen_rows fills bD
    for (int q = 0; q < g.nrhs; ++q) {
      const int64_t e = lin * g.nrhs + q;
      const double v = b_dtype == KR_F32 ? (double)((const float*)b)[e] : ((const double*)b)[e];
      bD[j * g.nrhs + q] = v;
      bad |= !isfinite(v);
    }
  }
  if (bad) atomicOr(flags, KR_FLAG_NONFINITE);
}

// ---------------------------------------------------------------------------
// Reordered modes: a prod(R) x nrhs tensor between the caller's mode order and
// the tree's.  to_tree: dst[r'][q] = src[r][q]; else dst[r][q] = src[r'][q], where
// r' is the tree-order multi-index (r'_n = r_{orig[n]}).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_permute_modes(Geom g, const double* __restrict__ src,
                                                       double* __restrict__ dst, int to_tree) {
  const int N = g.N, nrhs = g.nrhs;
  const int64_t total = g.Rtot * nrhs;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t rt = e / nrhs;
    const int q = (int)(e - rt * nrhs);
    int r[KR_MAXN];
    int64_t rem = rt;
    for (int n = N - 1; n >= 0; --n) {
      r[n] = (int)(rem % g.R[n]);
      rem /= g.R[n];
    }
    int64_t lin = 0;
    for (int o = 0; o < N; ++o) lin = lin * g.R[g.inv[o]] + r[g.inv[o]];
    if (to_tree) dst[e] = src[lin * nrhs + q];
    else dst[lin * nrhs + q] = src[e];
  }
}

// ---------------------------------------------------------------------------
// Implicit response b = K X_true + sigma E, formed at the distinct rows only.
// K X_true at a sampled row is the same Kronecker-row product as K~x in the
// iteration, taken down the sample tree with X_true in place of x.
// ---------------------------------------------------------------------------

// Forward level k applied to X_true:
// P_k[s][cq] = sum_r A_{k-1}[i_k(s)][r] P_{k-1}[parent(s)][r][cq], P_0 = X_true.
__global__ void __launch_bounds__(256) k_gen_level(Geom g, Tree tr, int k, const double* __restrict__ Pp,
                                                   double* __restrict__ Po) {
  const int64_t S = tr.cnt[k];
  const int64_t W = g.rsuf[k] * g.nrhs, Wp = g.rsuf[k - 1] * g.nrhs;
  const int Rk = g.R[k - 1];
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < S * W;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = e / W, cq = e - s * W;
    const int64_t p = k == 1 ? 0 : tr.parent[k][s];
    const double* __restrict__ a = tr.arow[k] + s * Rk;
    const double* __restrict__ src = Pp + p * Wp + cq;
    double acc = 0.0;
    for (int r = 0; r < Rk; ++r) acc = fma(a[r], src[(int64_t)r * W], acc);
    Po[e] = acc;
  }
}

// Standard normal E[i][q]: Box-Muller on the first two words of Philox4x64-10
// with counter (i, q, 0, 0) and key (seed, stream).
__device__ __forceinline__ double gen_normal(uint64_t i, uint64_t q, uint64_t seed, uint64_t stream) {
  const u64x4 w = philox4x64_10(i, q, 0ull, 0ull, seed, stream);
  const double u1 = (double)((w.v[0] >> 11) + 1ull) * 0x1p-53;
  const double u2 = (double)(w.v[1] >> 11) * 0x1p-53;
  const double two_pi = 6.283185307179586;
  return sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
}

// b~_j[q] = (K X_true)[i_j][q] + sigma E[i_j][q] for every distinct row j: the
// last two tree levels contracted from P_{N-2} (X_true itself when N <= 2).
__global__ void __launch_bounds__(256) k_gen_rows(Geom g, Tree tr, const double* __restrict__ Pn2, double sigma,
                                                  uint64_t seed, uint64_t stream, double* __restrict__ bD,
                                                  int32_t* __restrict__ flags) {
  const int N = g.N, nrhs = g.nrhs;
  const int64_t total = tr.cnt[N] * nrhs;
  const int RL = g.R[N - 1];
  const int RP = N >= 2 ? g.R[N - 2] : 1;
  int bad = 0;
  // one thread per (row j, rhs q)
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / nrhs;
    const int q = (int)(e - j * nrhs);
    const uint64_t key = tr.rkey[j];
    int64_t lin = 0;   // K's row index in the caller's mode order
    for (int o = 0; o < N; ++o) {
      const int n = g.inv[o];
      lin = lin * g.I[n] + (int64_t)((key >> g.shift[n]) & ((1ull << g.bits[n]) - 1ull));
    }
    const double* __restrict__ aL = tr.arow[N] + j * RL;
    double y = 0.0;
    if (N == 1) {
      for (int r = 0; r < RL; ++r) y = fma(aL[r], Pn2[(int64_t)r * nrhs + q], y);
    } else {
      const int64_t s = tr.parent[N][j];
      const double* __restrict__ aP = tr.arow[N - 1] + s * RP;
      const int64_t base = (N >= 3 ? (int64_t)tr.parent[N - 1][s] : 0) * g.rsuf[N - 2] * nrhs + q;
      for (int r1 = 0; r1 < RP; ++r1) {
        double t = 0.0;
        for (int r2 = 0; r2 < RL; ++r2) t = fma(aL[r2], Pn2[base + ((int64_t)r1 * RL + r2) * nrhs], t);
        y = fma(aP[r1], t, y);
      }
    }
    const double v = y + sigma * gen_normal((uint64_t)lin, (uint64_t)q, seed, stream);
    bD[j * nrhs + q] = v;
    bad |= !isfinite(v);
  }
  if (bad) atomicOr(flags, KR_FLAG_NONFINITE);
}

}  // namespace kr
