// Particle binning by grid tile and the LDS-privatised charge deposition of the tracking loop.
//
// Every step the particles are counting-sorted by the tile of their stencil's first node
// (tiles of T_x x T_y x T_z cells, at most 4096 tiles).  Particles move several cells per step,
// so the order is rebuilt each step; the previous step's order keeps every pass coherent:
//   k_key_hist     tile key of each particle (4 B) and a block-privatised histogram in LDS,
//                  flushed with one global atomic per non-empty bin;
//   k_build_chunks exclusive scan of the tile counts (sort offsets) and the work list of
//                  (tile, begin, end) chunks of at most `chunk` particles for the deposit;
//   k_scatter      moves phase space and particle ids to their sorted slots: each block
//                  counts its keys in LDS, reserves one contiguous range per key with a single
//                  global atomic, then ranks its particles with LDS atomics, so particles of one
//                  key leave a block as one contiguous run (first step of a call, where the
//                  caller's order is unrelated to the tiles);
//   k_scatter_perm the same ranking without moving anything: the source index of every sorted
//                  slot (4 B per particle instead of 104).  Later steps read the particles
//                  through it, and the gather-kick writes the new state in sorted order, so the
//                  phase space crosses HBM once per step fewer;
//   k_deposit_tiles each workgroup takes a chunk, accumulates the (T + S)^3 window of its tile
//                  with 64-bit fixed-point LDS atomics, and adds the non-zero window entries to
//                  the tile's own 64-bit integer window in HBM with one integer atomic each;
//   k_tile_reduce  forms the charge grid from the tiles' integer windows in a fixed order, so
//                  the grid depends neither on the particle order nor on that of the atomics;
//   k_gkd_tiles    the gather, kick and push of a chunk from its tile's E' window in LDS,
//                  reading through the ranking and writing the new state in sorted order.
#include "device_common.hpp"
#include "internal.hpp"

namespace pic {

namespace {

constexpr int kBlk = 256;
constexpr int kItems = 4096;               // particles per block in key_hist / scatter
constexpr int kPer = kItems / kBlk;         // 16 per thread

// stencil base node along one axis: the very function the deposit and gather kernels use
template <int S>
__device__ __forceinline__ int base_node(double u, int n) {
  double w[S + 1];
  return stencil<S>(u, n, w);
}

template <int S>
__device__ __forceinline__ uint32_t tile_key(double x, double y, double z, const double* o,
                                             const double* ih, const Consts& c,
                                             const SortPlan& sp) {
  int bx = base_node<S>((x - o[0]) * ih[0], c.nx);
  int by = base_node<S>((y - o[1]) * ih[1], c.ny);
  int bz = base_node<S>((z - o[2]) * ih[2], c.nz);
  return (uint32_t)(((bz / sp.T[2]) * sp.NT[1] + (by / sp.T[1])) * sp.NT[0] + (bx / sp.T[0]));
}

template <int S>
__device__ __forceinline__ void key_hist_body(const double* __restrict__ X,
                                                   const Geom* __restrict__ g, Consts c,
                                                   SortPlan sp, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ hist, int blk, int nblk) {
  __shared__ uint32_t lh[kMaxTiles];
  if (g->status) return;
  const double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
  const double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
  for (int t = threadIdx.x; t < sp.ntiles; t += kBlk) lh[t] = 0u;
  __syncthreads();
  const int64_t n = c.n;
  const int64_t base = (int64_t)blk * kItems;
  for (int k = 0; k < kPer; ++k) {
    int64_t i = base + k * kBlk + threadIdx.x;
    if (i < n) {
      uint32_t key = tile_key<S>(X[i], X[2 * n + i], X[4 * n + i], o, ih, c, sp);
      keys[i] = key;
      atomicAdd(&lh[key], 1u);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < sp.ntiles; t += kBlk)
    if (lh[t]) atomicAdd(&hist[t], lh[t]);
}

template <int S>
__global__ __launch_bounds__(kBlk) void k_key_hist(const double* __restrict__ X,
                                                   const Geom* __restrict__ g, Consts c,
                                                   SortPlan sp, uint32_t* __restrict__ keys,
                                                   uint32_t* __restrict__ hist) {
  key_hist_body<S>(X, g, c, sp, keys, hist, blockIdx.x, gridDim.x);
}

// Block-wide exclusive scan of per-thread values (1024 threads).
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t add = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  uint32_t incl = sh[t];
  *total = sh[1023];
  __syncthreads();
  return incl - v;
}

// one block of 1024 threads; each thread owns 4 consecutive tiles
__device__ __forceinline__ void build_chunks_body(const Geom* __restrict__ g, SortPlan sp,
                                                  uint32_t* __restrict__ hist,
                                                  uint32_t* __restrict__ cursor,
                                                  int4* __restrict__ chunks,
                                                  uint32_t* __restrict__ nchunks) {
  __shared__ uint32_t sh[1024];
  if (g->status) {
    if (threadIdx.x == 0) *nchunks = 0u;
    return;
  }
  const int t0 = threadIdx.x * 4;
  uint32_t cnt[4], nck[4], sc = 0, sk = 0;
  for (int q = 0; q < 4; ++q) {
    int t = t0 + q;
    cnt[q] = t < sp.ntiles ? hist[t] : 0u;
    nck[q] = (cnt[q] + sp.chunk - 1) / sp.chunk;
    sc += cnt[q];
    sk += nck[q];
  }
  uint32_t tot_c, tot_k;
  uint32_t off = block_exclusive_scan(sc, sh, &tot_c);
  uint32_t coff = block_exclusive_scan(sk, sh, &tot_k);
  for (int q = 0; q < 4; ++q) {
    int t = t0 + q;
    if (t < sp.ntiles) {
      cursor[t] = off;
      hist[t] = 0u;  // ready for the next step
      for (uint32_t k = 0; k < nck[q]; ++k) {
        uint32_t b = off + k * sp.chunk;
        uint32_t e = b + sp.chunk < off + cnt[q] ? b + sp.chunk : off + cnt[q];
        chunks[coff + k] = make_int4(t, (int)b, (int)e, (int)cnt[q]);  // w: the tile's count
      }
    }
    off += cnt[q];
    coff += nck[q];
  }
  if (threadIdx.x == 0) *nchunks = tot_k;
}

__global__ __launch_bounds__(1024) void k_build_chunks(const Geom* __restrict__ g, SortPlan sp,
                                                       uint32_t* __restrict__ hist,
                                                       uint32_t* __restrict__ cursor,
                                                       int4* __restrict__ chunks,
                                                       uint32_t* __restrict__ nchunks) {
  build_chunks_body(g, sp, hist, cursor, chunks, nchunks);
}

// In-place exclusive scan of a[0..count) (count <= kMaxTiles) by one block of NT threads;
// each thread owns a run of consecutive entries.
template <int NT>
__device__ void block_exclusive_scan_lds(uint32_t* a, int count) {
  __shared__ uint32_t part[NT];
  const int per = (count + NT - 1) / NT;
  const int b = threadIdx.x * per;
  const int e = min(b + per, count);
  uint32_t sum = 0;
  for (int t = b; t < e; ++t) sum += a[t];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < NT; off <<= 1) {
    const uint32_t add = threadIdx.x >= off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - sum;
  for (int t = b; t < e; ++t) {
    const uint32_t v = a[t];
    a[t] = run;
    run += v;
  }
  __syncthreads();
}

// LDS atomic add of 1 per active lane to lh[key], aggregated over the wave: one atomic per
// distinct key among the active lanes (their count), each lane getting the value it would
// have had from its own atomic in lane order.  Called by all lanes of the wave (the loop is
// wave-uniform).  After the first step of a call the particles arrive in the previous step's
// tile order, so a wave holds only a few distinct keys and the same-address atomics that
// would serialise lane by lane collapse into one per key.
__device__ __forceinline__ uint32_t wave_aggregated_add(uint32_t* lh, uint32_t key, bool active) {
  const int lane = (int)__lane_id();
  const uint64_t below = (1ull << lane) - 1ull;
  uint64_t todo = __ballot(active);
  uint32_t out = 0u;
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;  // wave-uniform
    const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, leader);
    const uint64_t grp = todo & __ballot(key == k0);
    uint32_t b = 0u;
    if (lane == leader) b = atomicAdd(&lh[k0], (uint32_t)__popcll(grp));
    b = (uint32_t)__builtin_amdgcn_readlane((int)b, leader);
    if ((grp >> lane) & 1ull) out = b + (uint32_t)__popcll(grp & below);
    todo &= ~grp;
  }
  return out;
}

// Counting-sort scatter of one block of kItems particles, staged: the block ranks its items by
// key in LDS (local offsets by a scan of its key counts, one global atomic per key present to
// reserve the key's run in the output), then moves each row through LDS in ranked order, so
// every key's run leaves the block as consecutive lanes writing consecutive addresses.  Used
// where the input order is unrelated to the keys (the caller's order, the id buckets of the
// final reordering): there it writes 3.6 times fewer bytes than the direct form.
__device__ __forceinline__ void scatter_staged_body(const double* __restrict__ A,
                                                  const uint32_t* __restrict__ idA,
                                                  const uint32_t* __restrict__ keys,
                                                  const Geom* __restrict__ g, int64_t n,
                                                  int ntiles, uint32_t* __restrict__ cursor,
                                                  double* __restrict__ B,
                                                  uint32_t* __restrict__ idB, int blk, int nblk) {
  // cur/delta (ranking) and the row buffer share storage
  __shared__ __align__(16) unsigned char stage[2 * kMaxTiles * sizeof(uint32_t)];
  __shared__ uint32_t dest[kItems];
  static_assert(kItems * sizeof(double) <= sizeof(stage), "row buffer exceeds its storage");
  uint32_t* cur = reinterpret_cast<uint32_t*>(stage);
  uint32_t* delta = cur + kMaxTiles;
  double* rowbuf = reinterpret_cast<double*>(stage);
  uint32_t* idbuf = reinterpret_cast<uint32_t*>(stage);
  if (g->status) return;
  const int64_t base = (int64_t)blk * kItems;
  const int m = (int)min((int64_t)kItems, n - base);
  for (int t = threadIdx.x; t < ntiles; t += kBlk) cur[t] = 0u;
  __syncthreads();
  uint32_t key[kPer];
  for (int k = 0; k < kPer; ++k) {
    const int l = k * kBlk + threadIdx.x;
    key[k] = l < m ? keys[base + l] : 0u;
    if (l < m) atomicAdd(&cur[key[k]], 1u);
  }
  __syncthreads();
  // reserve each present key's run in the output
  for (int t = threadIdx.x; t < ntiles; t += kBlk) {
    const uint32_t c = cur[t];
    delta[t] = c ? atomicAdd(&cursor[t], c) : 0u;
  }
  __syncthreads();
  block_exclusive_scan_lds<kBlk>(cur, ntiles);  // cur[t] = local offset of key t
  for (int t = threadIdx.x; t < ntiles; t += kBlk) delta[t] -= cur[t];
  __syncthreads();
  uint32_t slot[kPer];
  for (int k = 0; k < kPer; ++k) {
    const int l = k * kBlk + threadIdx.x;
    if (l < m) {
      slot[k] = atomicAdd(&cur[key[k]], 1u);
      dest[slot[k]] = delta[key[k]] + slot[k];
    }
  }
  __syncthreads();
  const int rows = idA ? 7 : 6;  // the ids travel as a seventh row when there are any
  for (int r = 0; r < rows; ++r) {
    for (int k = 0; k < kPer; ++k) {
      const int l = k * kBlk + threadIdx.x;
      if (l < m) {
        if (r < 6)
          rowbuf[slot[k]] = A[r * n + base + l];
        else
          idbuf[slot[k]] = idA[base + l];
      }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < m; q += kBlk) {
      const uint32_t d = dest[q];
      if (d < (uint64_t)n) {  // always true for a consistent histogram; keeps writes in bounds
        if (r < 6)
          B[r * n + d] = rowbuf[q];
        else
          idB[d] = idbuf[q];
      }
    }
    __syncthreads();
  }
}

// Counting-sort scatter of one block of kItems particles, written straight from registers: the
// block counts its keys in LDS, reserves one run per key with a global atomic, and ranks its
// particles with LDS atomics.  When the input is already close to the key order (the previous
// step's binning), the lanes of a wave mostly share a key and get consecutive slots, so the
// writes coalesce without staging.
__device__ __forceinline__ void scatter_direct_body(const double* __restrict__ A,
                                                  const uint32_t* __restrict__ idA,
                                                  const uint32_t* __restrict__ keys,
                                                  const Geom* __restrict__ g, int64_t n,
                                                  int ntiles, uint32_t* __restrict__ cursor,
                                                  double* __restrict__ B,
                                                  uint32_t* __restrict__ idB, int blk, int nblk) {
  __shared__ uint32_t lh[kMaxTiles];
  if (g->status) return;
  for (int t = threadIdx.x; t < ntiles; t += kBlk) lh[t] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blk * kItems;
  uint32_t key[kPer];
  for (int k = 0; k < kPer; ++k) {
    int64_t i = base + k * kBlk + threadIdx.x;
    key[k] = i < n ? keys[i] : 0u;
    if (i < n) atomicAdd(&lh[key[k]], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < ntiles; t += kBlk)
    if (lh[t]) lh[t] = atomicAdd(&cursor[t], lh[t]);
  __syncthreads();
  for (int k = 0; k < kPer; ++k) {
    int64_t i = base + k * kBlk + threadIdx.x;
    if (i < n) {
      uint32_t pos = atomicAdd(&lh[key[k]], 1u);
      if (pos < (uint64_t)n) {  // always true for a consistent histogram; keeps writes in bounds
        for (int r = 0; r < 6; ++r) B[r * n + pos] = A[r * n + i];
        if (idA) idB[pos] = idA[i];
      }
    }
  }
}

// Ranking of one block of kItems particles as in the direct form, writing only the source
// index of each slot: perm[slot] = i.
__device__ __forceinline__ void scatter_perm_body(const uint32_t* __restrict__ keys,
                                                  const Geom* __restrict__ g, int64_t n,
                                                  int ntiles, uint32_t* __restrict__ cursor,
                                                  uint32_t* __restrict__ perm, int blk) {
  __shared__ uint32_t lh[kMaxTiles];
  if (g->status) return;
  for (int t = threadIdx.x; t < ntiles; t += kBlk) lh[t] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blk * kItems;
  // all of the thread's keys are loaded before the first (wave-uniform, branching) histogram
  // add, so that the loads overlap instead of each waiting behind the previous add
  uint32_t key[kPer];
  for (int k = 0; k < kPer; ++k) {
    int64_t i = base + k * kBlk + threadIdx.x;
    key[k] = i < n ? keys[i] : 0u;
  }
  for (int k = 0; k < kPer; ++k)
    (void)wave_aggregated_add(lh, key[k], base + k * kBlk + threadIdx.x < n);
  __syncthreads();
  for (int t = threadIdx.x; t < ntiles; t += kBlk)
    if (lh[t]) lh[t] = atomicAdd(&cursor[t], lh[t]);
  __syncthreads();
  for (int k = 0; k < kPer; ++k) {
    int64_t i = base + k * kBlk + threadIdx.x;
    const uint32_t pos = wave_aggregated_add(lh, key[k], i < n);
    // in bounds for a consistent histogram
    if (i < n && pos < (uint64_t)n) perm[pos] = (uint32_t)i;
  }
}

__global__ __launch_bounds__(kBlk) void k_scatter_perm(const uint32_t* __restrict__ keys,
                                                       const Geom* __restrict__ g, int64_t n,
                                                       int ntiles, uint32_t* __restrict__ cursor,
                                                       uint32_t* __restrict__ perm) {
  scatter_perm_body(keys, g, n, ntiles, cursor, perm, blockIdx.x);
}

template <bool STAGED>
__device__ __forceinline__ void scatter_body(const double* __restrict__ A,
                                             const uint32_t* __restrict__ idA,
                                             const uint32_t* __restrict__ keys,
                                             const Geom* __restrict__ g, int64_t n, int ntiles,
                                             uint32_t* __restrict__ cursor, double* __restrict__ B,
                                             uint32_t* __restrict__ idB, int blk, int nblk) {
  if constexpr (STAGED)
    scatter_staged_body(A, idA, keys, g, n, ntiles, cursor, B, idB, blk, nblk);
  else
    scatter_direct_body(A, idA, keys, g, n, ntiles, cursor, B, idB, blk, nblk);
}

template <bool STAGED>
__global__ __launch_bounds__(kBlk) void k_scatter(const double* __restrict__ A,
                                                  const uint32_t* __restrict__ idA,
                                                  const uint32_t* __restrict__ keys,
                                                  const Geom* __restrict__ g, int64_t n,
                                                  int ntiles, uint32_t* __restrict__ cursor,
                                                  double* __restrict__ B,
                                                  uint32_t* __restrict__ idB) {
  scatter_body<STAGED>(A, idA, keys, g, n, ntiles, cursor, B, idB, blockIdx.x, gridDim.x);
}

// The staged scatter over wide blocks, for inputs whose order is unrelated to the keys (the
// caller's order on a call's first step, the id buckets of the final reordering).  A block of
// kWBlk threads takes kWItems particles, four times the items of k_scatter<true>, so that every
// key's run in the output is four times longer (at 2048 tiles about 8 particles, 64 B per row,
// instead of 2): the runs' writes then fill whole 64-byte pieces of memory instead of a
// fraction of one.  The ranking is that of the staged form; the rows then move through a
// kWHalf-slot LDS buffer in two halves of the ranked slots, each item's value read from HBM in
// the half its slot falls in.
constexpr int kWBlk = 1024;
constexpr int kWPer = 16;
constexpr int kWItems = kWBlk * kWPer;  // 16384
constexpr int kWHalf = kWItems / 2;     // slots staged per pass

__global__ __launch_bounds__(kWBlk) void k_scatter_wide(const double* __restrict__ A,
                                                        const uint32_t* __restrict__ idA,
                                                        const uint32_t* __restrict__ keys,
                                                        const Geom* __restrict__ g, int64_t n,
                                                        int ntiles, uint32_t* __restrict__ cursor,
                                                        double* __restrict__ B,
                                                        uint32_t* __restrict__ idB) {
  // cur/delta (ranking, 2 x kMaxTiles words) and the row buffer (kWHalf doubles) share storage
  __shared__ __align__(16) unsigned char stage[kWHalf * sizeof(double)];
  __shared__ uint32_t dest[kWItems];
  static_assert(2 * kMaxTiles * sizeof(uint32_t) <= sizeof(stage), "ranking exceeds storage");
  uint32_t* cur = reinterpret_cast<uint32_t*>(stage);
  uint32_t* delta = cur + kMaxTiles;
  double* rowbuf = reinterpret_cast<double*>(stage);
  uint32_t* idbuf = reinterpret_cast<uint32_t*>(stage);
  if (g->status) return;
  const int64_t base = (int64_t)blockIdx.x * kWItems;
  const int m = (int)min((int64_t)kWItems, n - base);
  for (int t = threadIdx.x; t < ntiles; t += kWBlk) cur[t] = 0u;
  __syncthreads();
  uint32_t key[kWPer];
  for (int k = 0; k < kWPer; ++k) {
    const int l = k * kWBlk + threadIdx.x;
    key[k] = l < m ? keys[base + l] : 0u;
  }
  for (int k = 0; k < kWPer; ++k)
    if (k * kWBlk + (int)threadIdx.x < m) atomicAdd(&cur[key[k]], 1u);
  __syncthreads();
  // reserve each present key's run in the output
  for (int t = threadIdx.x; t < ntiles; t += kWBlk) {
    const uint32_t c = cur[t];
    delta[t] = c ? atomicAdd(&cursor[t], c) : 0u;
  }
  __syncthreads();
  block_exclusive_scan_lds<kWBlk>(cur, ntiles);  // cur[t] = local offset of key t
  for (int t = threadIdx.x; t < ntiles; t += kWBlk) delta[t] -= cur[t];
  __syncthreads();
  uint32_t slot[kWPer];
  for (int k = 0; k < kWPer; ++k) {
    const int l = k * kWBlk + threadIdx.x;
    slot[k] = 0u;
    if (l < m) {
      slot[k] = atomicAdd(&cur[key[k]], 1u);
      dest[slot[k]] = delta[key[k]] + slot[k];
    }
  }
  __syncthreads();  // the ranking's words are dead from here: the row buffer takes them over
  const int rows = idA ? 7 : 6;  // the ids travel as a seventh row when there are any
  for (int r = 0; r < rows; ++r) {
    for (int h = 0; h < 2; ++h) {
      const uint32_t lo = (uint32_t)(h * kWHalf);
      for (int k = 0; k < kWPer; ++k) {
        const int l = k * kWBlk + threadIdx.x;
        if (l < m && slot[k] - lo < (uint32_t)kWHalf) {
          if (r < 6)
            rowbuf[slot[k] - lo] = A[r * n + base + l];
          else
            idbuf[slot[k] - lo] = idA[base + l];
        }
      }
      __syncthreads();
      const int cnt = min(kWHalf, m - (int)lo);
      for (int q = threadIdx.x; q < cnt; q += kWBlk) {
        const uint32_t d = dest[lo + q];
        if (d < (uint64_t)n) {  // always true for a consistent histogram; keeps writes in bounds
          if (r < 6)
            B[r * n + d] = rowbuf[q];
          else
            idB[d] = idbuf[q];
        }
      }
      __syncthreads();
    }
  }
}

template <typename T>
__device__ __forceinline__ void add_global(T* p, T v) {
  unsafeAtomicAdd(p, v);
}

// Charge of one chunk in its tile's (T + S)^3 window, accumulated in LDS as 64-bit fixed point:
// every contribution q_m w is scaled by a power of two 2^k chosen from the whole charge of the
// chunk's tile, |q_m| * count_tile 2^k <= 2^62 (no overflow in any node, whatever the order;
// the same k for all chunks of the tile), with a single contribution below 2^50, rounded to
// the nearest integer (error below 2^-(k+1) |q_m|) and added with integer LDS atomics, which
// are exact, so the window sum does not depend on the order of the lanes.  Integer LDS atomics
// also run faster here than floating-point ones (1.13 ms against 1.85 ms with float64 and 13 ms
// with float32 atomics for 1e8 TSC particles on MI355X).  The non-zero window entries are then
// added, still as integers, to the tile's own window in tacc (tacc[t nw + w], one 64-bit
// integer atomic each, exact in any order); the tile's exponent goes to tscale[t], and
// k_tile_reduce forms the grid, which then depends neither on the order of the particles nor
// on that of the atomics.
template <int S, typename T, bool PERM>
__device__ __forceinline__ void deposit_tiles_body(const double* __restrict__ B,
                                                        const uint32_t* __restrict__ perm,
                                                        const Geom* __restrict__ g, Consts c,
                                                        SortPlan sp,
                                                        const int4* __restrict__ chunks,
                                                        const uint32_t* __restrict__ nchunks,
                                                        T* __restrict__ rho, int blk, int nblk,
                                                        unsigned long long* __restrict__ tacc,
                                                        int* __restrict__ tscale) {
  extern __shared__ unsigned char smem_raw[];
  unsigned long long* win = reinterpret_cast<unsigned long long*>(smem_raw);
  if (g->status) return;
  const double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
  const double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
  const int Wx = sp.T[0] + S, Wy = sp.T[1] + S, Wz = sp.T[2] + S;
  const int nw = Wx * Wy * Wz;
  int rowoff[S + 1][S + 1];  // window offset of stencil row (a, b)
  for (int a = 0; a <= S; ++a)
    for (int b = 0; b <= S; ++b) rowoff[a][b] = (a * Wy + b) * Wx;
  const int64_t n = c.n;
  bool bin_fault = false;
  const uint32_t nck = *nchunks;
  for (uint32_t ci = blk; ci < nck; ci += nblk) {
    const int4 ch = chunks[ci];
    const int t = ch.x;
    const int tx = t % sp.NT[0], ty = (t / sp.NT[0]) % sp.NT[1], tz = t / (sp.NT[0] * sp.NT[1]);
    const int ox = tx * sp.T[0], oy = ty * sp.T[1], oz = tz * sp.T[2];
    // scale 2^k with |q_m| * count * 2^k <= 2^62 (no node overflows) and |q_m| 2^k <= 2^50
    // (every scaled contribution converts exactly below); a zero charge gives zero
    const double qa = fabs(c.q_macro);
    const double qc = qa * (double)ch.w;  // the tile's particle count
    const int k = qc > 0.0 ? min(62 - max(ilogb(qc) + 1, -960), 50 - max(ilogb(qa) + 1, -960)) : 0;
    const double qs = c.q_macro * ldexp(1.0, k);
    if (threadIdx.x == 0) tscale[t] = k;  // every chunk of the tile writes the same k
    for (int w = threadIdx.x; w < nw; w += (int)blockDim.x) win[w] = 0ull;
    __syncthreads();
    // Software-pipelined over the lane's slots i, i + stride, ... in pairs (a, b): before the
    // atomics of one slot the positions of the lane's next slot and the index of the slot after
    // that are loaded.  No branch surrounds these loads (slot indices are clamped into the chunk
    // and particle indices into [0, n), and a result is used only where it is valid), so the
    // waits for them fall at their first use and they stay in flight during the LDS atomics; a
    // load inside a branch makes the join wait for every load the wave has issued.  Slot i
    // holds particle perm[i] of B (B itself in slot order without a permutation); an index past
    // n, impossible for a consistent ranking, is flagged and its particle skipped.
    const int64_t stride = (int)blockDim.x;
    const int64_t last = ch.z - 1;  // a work item holds at least one slot
    auto index_of = [&](int64_t j) -> int64_t {
      j = j < last ? j : last;
      if constexpr (PERM) return (int64_t)perm[j];
      return j;
    };
    auto load_pos = [&](int64_t r, double* p) {
      const int64_t q = r < n ? r : 0;
      p[0] = B[q];
      p[1] = B[2 * n + q];
      p[2] = B[4 * n + q];
    };
    auto deposit_one = [&](const double* p, int64_t r) {
      const bool valid = r < n;
      if (!valid) bin_fault = true;
      double wx[S + 1], wy[S + 1], wz[S + 1];
      const int bx = stencil<S>((p[0] - o[0]) * ih[0], c.nx, wx);
      const int by = stencil<S>((p[1] - o[1]) * ih[1], c.ny, wy);
      const int bz = stencil<S>((p[2] - o[2]) * ih[2], c.nz, wz);
      const int lx = bx - ox, ly = by - oy, lz = bz - oz;
      const bool inside = lx >= 0 && lx < sp.T[0] && ly >= 0 && ly < sp.T[1] && lz >= 0 &&
                          lz < sp.T[2];
      // the binning put the particle in the chunk's tile with this very stencil function, so
      // its stencil lies in the window; a violation is a library fault, flagged as the
      // gather-kick flags it (PIC_EINTERNAL), and the particle is not deposited
      if (valid && !inside) bin_fault = true;
      if (valid && inside) {
        // q_m 2^k w rounded to the nearest integer by one fused multiply-add with 1.5 2^52
        // (the sum then has the integer in its low mantissa bits, |value| < 2^51), read back
        // as a two's-complement int64 by subtracting the constant's bit pattern
        constexpr double kMagic = 6755399441055744.0;  // 1.5 * 2^52
        constexpr unsigned long long kMagicBits = 0x4338000000000000ull;
        unsigned long long* w0 = win + (lz * Wy + ly) * Wx + lx;
        for (int a = 0; a <= S; ++a) {
          const double wzs = qs * wz[a];
          for (int b = 0; b <= S; ++b) {
            const double wzy = wzs * wy[b];
            unsigned long long* row = w0 + rowoff[a][b];
            for (int q = 0; q <= S; ++q) {
              const double d = __builtin_fma(wzy, wx[q], kMagic);
              atomicAdd(row + q, (unsigned long long)__double_as_longlong(d) - kMagicBits);
            }
          }
        }
      }
    };
    int64_t i = ch.y + threadIdx.x;
    int64_t ra = index_of(i), rb = index_of(i + stride);
    double pa[3], pb[3];
    load_pos(ra, pa);
    for (; i < ch.z; i += 2 * stride) {
      const int64_t ra2 = index_of(i + 2 * stride);
      load_pos(rb, pb);
      deposit_one(pa, ra);  // slot i
      const int64_t rb2 = index_of(i + 3 * stride);
      load_pos(ra2, pa);
      if (i + stride < ch.z) deposit_one(pb, rb);  // slot i + stride
      ra = ra2;
      rb = rb2;
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nw; w += (int)blockDim.x) {
      const long long v = (long long)win[w];
      int wx_ = w % Wx, wy_ = (w / Wx) % Wy, wz_ = w / (Wx * Wy);
      int gx = ox + wx_, gy = oy + wy_, gz = oz + wz_;
      if (v != 0 && gx < c.nx && gy < c.ny && gz < c.nz)
        atomicAdd(&tacc[(int64_t)t * nw + w], (unsigned long long)v);
    }
    __syncthreads();
  }
  if (bin_fault) atomicCAS(const_cast<int*>(&g->status), 0, -7);
}

// The charge grid from the tiles' integer windows: every node adds, in ascending tile order
// (z, then y, then x), the windows of the tiles that cover it, each scaled back by its tile's
// 2^-k, to what the deposit's direct path put there, and clears the entries it read, so that
// tacc is zero again for the next step (entries outside the grid are never written).
template <int S, typename T>
__device__ __forceinline__ void tile_reduce_body(const Geom* __restrict__ g, Consts c,
                                                 SortPlan sp,
                                                 unsigned long long* __restrict__ tacc,
                                                 const int* __restrict__ tscale,
                                                 T* __restrict__ rho, int blk, int nblk) {
  if (g->status) return;
  const int Wx = sp.T[0] + S, Wy = sp.T[1] + S, Wz = sp.T[2] + S;
  const int64_t nw = (int64_t)Wx * Wy * Wz;
  const int64_t total = (int64_t)c.nx * c.ny * c.nz;
  for (int64_t node = blk * 256ll + threadIdx.x; node < total; node += (int64_t)nblk * 256) {
    const int gx = (int)(node % c.nx), gy = (int)((node / c.nx) % c.ny),
              gz = (int)(node / ((int64_t)c.nx * c.ny));
    const int p[3] = {gx, gy, gz};
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {  // tiles whose window [t T, t T + T + S) holds p[a]
      hi[a] = min(p[a] / sp.T[a], sp.NT[a] - 1);
      lo[a] = hi[a];
      while (lo[a] > 0 && (lo[a] - 1) * sp.T[a] + sp.T[a] + S > p[a]) --lo[a];
    }
    double val = 0.0;
    for (int tz = lo[2]; tz <= hi[2]; ++tz)
      for (int ty = lo[1]; ty <= hi[1]; ++ty)
        for (int tx = lo[0]; tx <= hi[0]; ++tx) {
          const int t = (tz * sp.NT[1] + ty) * sp.NT[0] + tx;
          const int64_t w = ((int64_t)(gz - tz * sp.T[2]) * Wy + (gy - ty * sp.T[1])) * Wx +
                            (gx - tx * sp.T[0]);
          unsigned long long* e = &tacc[t * nw + w];
          const long long v = (long long)*e;
          if (v != 0) {
            val += ldexp((double)v, -tscale[t]);
            *e = 0ull;
          }
        }
    if (val != 0.0) rho[node] = (T)((double)rho[node] + val);
  }
}

template <int S, typename T>
__global__ __launch_bounds__(256) void k_tile_reduce(const Geom* __restrict__ g, Consts c,
                                                     SortPlan sp,
                                                     unsigned long long* __restrict__ tacc,
                                                     const int* __restrict__ tscale,
                                                     T* __restrict__ rho) {
  tile_reduce_body<S, T>(g, c, sp, tacc, tscale, rho, blockIdx.x, gridDim.x);
}

// Vector deposit e_c(node) = sum_i W(r_i - node) v_c,i of the binned rows (r_x, v_x, r_y, v_y,
// r_z, v_z) of B (the reverse sweep's transposed gather), one chunk per workgroup: three
// float64 LDS windows (the values have both signs), flushed with global atomics.
template <int S, typename T>
__device__ __forceinline__ void vdeposit_tiles_body(const double* __restrict__ B,
                                                    const Geom* __restrict__ g, Consts c,
                                                    SortPlan sp,
                                                    const int4* __restrict__ chunks,
                                                    const uint32_t* __restrict__ nchunks,
                                                    T* __restrict__ e, int blk, int nblk) {
  extern __shared__ unsigned char smem_raw[];
  double* win = reinterpret_cast<double*>(smem_raw);
  if (g->status) return;
  const double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
  const double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
  const int Wx = sp.T[0] + S, Wy = sp.T[1] + S, Wz = sp.T[2] + S;
  const int nw = Wx * Wy * Wz;
  const int64_t n = c.n;
  const int64_t ng = (int64_t)c.nx * c.ny * c.nz;
  const uint32_t nck = *nchunks;
  for (uint32_t ci = blk; ci < nck; ci += nblk) {
    const int4 ch = chunks[ci];
    const int t = ch.x;
    const int tx = t % sp.NT[0], ty = (t / sp.NT[0]) % sp.NT[1], tz = t / (sp.NT[0] * sp.NT[1]);
    const int ox = tx * sp.T[0], oy = ty * sp.T[1], oz = tz * sp.T[2];
    for (int w = threadIdx.x; w < 3 * nw; w += (int)blockDim.x) win[w] = 0.0;
    __syncthreads();
    for (int64_t i = ch.y + threadIdx.x; i < ch.z; i += (int)blockDim.x) {
      double wx[S + 1], wy[S + 1], wz[S + 1];
      const int bx = stencil<S>((B[i] - o[0]) * ih[0], c.nx, wx);
      const int by = stencil<S>((B[2 * n + i] - o[1]) * ih[1], c.ny, wy);
      const int bz = stencil<S>((B[4 * n + i] - o[2]) * ih[2], c.nz, wz);
      const double v[3] = {B[n + i], B[3 * n + i], B[5 * n + i]};
      const int lx = bx - ox, ly = by - oy, lz = bz - oz;
      const bool inside = lx >= 0 && lx < sp.T[0] && ly >= 0 && ly < sp.T[1] && lz >= 0 &&
                          lz < sp.T[2];
      for (int a = 0; a <= S; ++a)
        for (int b = 0; b <= S; ++b) {
          const double wzy = wz[a] * wy[b];
          for (int q = 0; q <= S; ++q) {
            const double w = wzy * wx[q];
            if (inside) {
              const int idx = ((lz + a) * Wy + (ly + b)) * Wx + (lx + q);
              for (int comp = 0; comp < 3; ++comp) atomicAdd(&win[comp * nw + idx], w * v[comp]);
            } else {
              const int64_t node = ((int64_t)(bz + a) * c.ny + (by + b)) * c.nx + (bx + q);
              for (int comp = 0; comp < 3; ++comp) add_global(&e[comp * ng + node], (T)(w * v[comp]));
            }
          }
        }
    }
    __syncthreads();
    for (int w = threadIdx.x; w < nw; w += (int)blockDim.x) {
      const int wx_ = w % Wx, wy_ = (w / Wx) % Wy, wz_ = w / (Wx * Wy);
      const int gx = ox + wx_, gy = oy + wy_, gz = oz + wz_;
      if (gx < c.nx && gy < c.ny && gz < c.nz) {
        const int64_t node = ((int64_t)gz * c.ny + gy) * c.nx + gx;
        for (int comp = 0; comp < 3; ++comp) {
          const double v = win[comp * nw + w];
          if (v != 0.0) add_global(&e[comp * ng + node], (T)v);
        }
      }
    }
    __syncthreads();
  }
}

template <int S, typename T>
__global__ __launch_bounds__(kMaxThreads) void k_vdeposit_tiles(const double* __restrict__ B,
                                                         const Geom* __restrict__ g, Consts c,
                                                         SortPlan sp,
                                                         const int4* __restrict__ chunks,
                                                         const uint32_t* __restrict__ nchunks,
                                                         T* __restrict__ e) {
  vdeposit_tiles_body<S, T>(B, g, c, sp, chunks, nchunks, e, blockIdx.x, gridDim.x);
}

template <int S, typename T>
__global__ __launch_bounds__(kMaxThreads) void k_deposit_tiles(const double* __restrict__ B,
                                                        const uint32_t* __restrict__ perm,
                                                        const Geom* __restrict__ g, Consts c,
                                                        SortPlan sp,
                                                        const int4* __restrict__ chunks,
                                                        const uint32_t* __restrict__ nchunks,
                                                        T* __restrict__ rho,
                                                        unsigned long long* __restrict__ tacc,
                                                        int* __restrict__ tscale) {
  // the permutation's presence as a template argument: a uniform branch around its loads
  // inside the loop would make the join wait for all of the wave's loads
  if (perm)
    deposit_tiles_body<S, T, true>(B, perm, g, c, sp, chunks, nchunks, rho, blockIdx.x,
                                   gridDim.x, tacc, tscale);
  else
    deposit_tiles_body<S, T, false>(B, nullptr, g, c, sp, chunks, nchunks, rho, blockIdx.x,
                                    gridDim.x, tacc, tscale);
}

// Fused second half of step j and first half of step j+1 on the sorted array, one chunk per
// workgroup: the (T + S)^3 window of E' around the chunk's tile is staged in LDS (coalesced
// rows), the particles gather from LDS, get the space-charge kick over L and the slice's second
// half map, then (has_next) the next slice's first half map (without DIAG the two as one
// product), and the box of the new positions is accumulated.  PERM false: B is in slot order and updated in place.  PERM true: slot i
// reads particle perm[i] of src (and its id) and writes the new state to slot i of B, so B
// leaves in sorted order.  The gather reads LDS only (a per-lane choice between LDS and global memory
// compiles to flat loads, which go through the vector memory pipeline); a stencil outside the
// window, impossible for a consistent binning, sets status -7 (PIC_EINTERNAL).
// PERM with a next step and no DIAG: the chunk's slots [begin, end) are refilled from both
// ends, the particles whose next kick-point position lies in the same tile of the current grid
// from the bottom and the others from the top (one LDS atomic per wavefront and end), so that
// the particles likely to change tile next step lie together in a short stretch of the order:
// neighbouring tiles then read them through the next permutation from fewer cache lines.
// DIAG: the particles' state at the end of the step (after the second half map, before the
// next first half map) is also summed into the block's partial moments, diag_part[blk * 27 +
// q]: 6 sums of d = v - shift and the 21 products d_a d_b (a <= b, row-major), with the
// 6-double shift read from diag_shift (close to the mean, so that the centred moments formed
// from these sums lose no digits).
template <int S, typename T, bool PERM, bool DIAG = false>
__device__ __forceinline__ void gkd_tiles_body(double* __restrict__ B,
                                                    const double* __restrict__ src,
                                                    const uint32_t* __restrict__ perm,
                                                    const uint32_t* __restrict__ idsrc,
                                                    uint32_t* __restrict__ iddst,
                                                    const Geom* __restrict__ g,
                                                    const T* __restrict__ E, Consts c,
                                                    SortPlan sp,
                                                    const int4* __restrict__ chunks,
                                                    const uint32_t* __restrict__ nchunks,
                                                    double L, const HalfMap& second,
                                                    int has_next, const HalfMap& first_next,
                                                    Box* box, int blk, int nblk,
                                                    double* __restrict__ diag_part = nullptr,
                                                    const double* __restrict__ diag_shift = nullptr) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ uint32_t s_up, s_down;  // the next free slot from either end of the chunk
  T* win = reinterpret_cast<T*>(smem_raw);
  if (g->status) return;
  const bool reorder = PERM && !DIAG && has_next;  // with DIAG it cost more time than it saved
  double sh[6], acc[DIAG ? kMomentSlots : 1];
  if constexpr (DIAG) {
    for (int r = 0; r < 6; ++r) sh[r] = diag_shift[r];
    for (int q = 0; q < kMomentSlots; ++q) acc[q] = 0.0;
  }
  // Without the moment sums, the slice's second half map and the next slice's first act back
  // to back on the kicked state: they are applied as their product (one matrix per plane, the
  // longitudinal coefficients summed), the same linear map in half the arithmetic and with few
  // enough uniform values to stay in scalar registers.
  // With the moment sums the two maps stay apart (the sums are taken between them), each in
  // matrix form.
  HalfMap maps, next_map;
  if constexpr (!DIAG) {
    maps = half_product(second, first_next, has_next != 0);
  } else {
    maps = half_product(second, second, false);
    next_map = half_product(first_next, first_next, false);
  }
  const double o[3] = {g->origin[0], g->origin[1], g->origin[2]};
  const double ih[3] = {g->inv_h[0], g->inv_h[1], g->inv_h[2]};
  const int Wx = sp.T[0] + S, Wy = sp.T[1] + S, Wz = sp.T[2] + S;
  const int nw = Wx * Wy * Wz;
  int rowoff[S + 1][S + 1];  // window offset of stencil row (a, b)
  for (int a = 0; a <= S; ++a)
    for (int b = 0; b <= S; ++b) rowoff[a][b] = (a * Wy + b) * Wx;
  const int64_t n = c.n;
  const int64_t plane = (int64_t)c.nx * c.ny * c.nz;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false, bin_fault = false;
  // the thread's first window entry and the block size, both split into (x, y, z) offsets
  const int w0x = (int)threadIdx.x % Wx, w0y = ((int)threadIdx.x / Wx) % Wy,
            w0z = (int)threadIdx.x / (Wx * Wy);
  const int stx = (int)blockDim.x % Wx, sty = ((int)blockDim.x / Wx) % Wy,
            stz = (int)blockDim.x / (Wx * Wy);
  const uint32_t nck = *nchunks;
  for (uint32_t ci = blk; ci < nck; ci += nblk) {
    const int4 ch = chunks[ci];
    const int t = ch.x;
    const int tx = t % sp.NT[0], ty = (t / sp.NT[0]) % sp.NT[1], tz = t / (sp.NT[0] * sp.NT[1]);
    const int ox = tx * sp.T[0], oy = ty * sp.T[1], oz = tz * sp.T[2];
    __syncthreads();  // the previous chunk's readers are done with the window and counters
    if (reorder && threadIdx.x == 0) {
      s_up = (uint32_t)ch.y;
      s_down = (uint32_t)ch.z;
    }
    // window entry w = (wz_ Wy + wy_) Wx + wx_, stepped by the block size with carries
    int wx_ = w0x, wy_ = w0y, wz_ = w0z;
    for (int w = threadIdx.x; w < nw; w += (int)blockDim.x) {
      int gx = ox + wx_, gy = oy + wy_, gz = oz + wz_;
      bool in = gx < c.nx && gy < c.ny && gz < c.nz;
      int64_t gi = ((int64_t)gz * c.ny + gy) * c.nx + gx;
      win[w] = in ? E[gi] : T(0);
      win[nw + w] = in ? E[plane + gi] : T(0);
      win[2 * nw + w] = in ? E[2 * plane + gi] : T(0);
      wx_ += stx;
      const int cx = wx_ >= Wx;
      wx_ -= cx ? Wx : 0;
      wy_ += sty + cx;
      const int cy = wy_ >= Wy;
      wy_ -= cy ? Wy : 0;
      wz_ += stz + cy;
    }
    __syncthreads();
    // every thread of the block runs the same number of rounds (the wavefront-wide slot
    // assignment below needs all lanes); lanes past the chunk's end are inactive
    for (int64_t ib = ch.y; ib < ch.z; ib += (int)blockDim.x) {
      const int64_t i = ib + threadIdx.x;
      const bool act = i < ch.z;
      double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
      int64_t i0 = i;
      if (act) {
        if constexpr (PERM) {
          i0 = perm[i];
          if (i0 >= n) {  // impossible for a consistent ranking; keeps the reads in bounds
            bin_fault = true;
            i0 = 0;
          }
          for (int r = 0; r < 6; ++r) v[r] = src[r * n + i0];
        } else {
          for (int r = 0; r < 6; ++r) v[r] = B[r * n + i];
        }
        double wx[S + 1], wy[S + 1], wz[S + 1];
        const int bx = stencil<S>((v[0] - o[0]) * ih[0], c.nx, wx);
        const int by = stencil<S>((v[2] - o[1]) * ih[1], c.ny, wy);
        const int bz = stencil<S>((v[4] - o[2]) * ih[2], c.nz, wz);
        // the binning put this particle in the chunk's tile, so its stencil lies in the window;
        // a violation is a library fault: flagged, and the indices clamped to stay in bounds
        int lx = bx - ox, ly = by - oy, lz = bz - oz;
        if (lx < 0 || lx >= sp.T[0] || ly < 0 || ly >= sp.T[1] || lz < 0 || lz >= sp.T[2]) {
          bin_fault = true;
          lx = min(max(lx, 0), sp.T[0] - 1);
          ly = min(max(ly, 0), sp.T[1] - 1);
          lz = min(max(lz, 0), sp.T[2] - 1);
        }
        T ex = 0, ey = 0, ez = 0;
        const T* w0 = win + (lz * Wy + ly) * Wx + lx;
        for (int a = 0; a <= S; ++a)
          for (int b = 0; b <= S; ++b) {
            const double wzy = wz[a] * wy[b];
            const T* row = w0 + rowoff[a][b];
            for (int q = 0; q <= S; ++q) {
              const T w = (T)(wzy * wx[q]);
              ex += w * row[q];
              ey += w * row[nw + q];
              ez += w * row[2 * nw + q];
            }
          }
        v[1] = v[1] + c.C * (double)ex * L;
        v[3] = v[3] + c.C * (double)ey * L;
        v[5] = v[5] + c.gamma * c.C * (double)ez * L;
        if constexpr (DIAG) {
          apply_matrix(maps, v, c.inv_gamma2);
          double d[6];
          for (int r = 0; r < 6; ++r) {
            d[r] = v[r] - sh[r];
            acc[r] += d[r];
          }
          int q = 6;
          for (int a = 0; a < 6; ++a)
            for (int b = a; b < 6; ++b) acc[q++] += d[a] * d[b];
          if (has_next) apply_matrix(next_map, v, c.inv_gamma2);
        } else {
          apply_matrix(maps, v, c.inv_gamma2);
        }
        if (has_next) {
          const double p[3] = {v[0], v[2], v[4]};
          for (int a = 0; a < 3; ++a) {
            bad |= !isfinite(p[a]);
            lo[a] = fmin(lo[a], p[a]);
            hi[a] = fmax(hi[a], p[a]);
          }
        }
      }
      int64_t slot = i;
      if (reorder) {
        // the particle keeps tile t when its new stencil base lies in t's node range: the same
        // test as tile_key(...) == t, without the divisions
        bool stay = false;
        if (act) {
          const int nx_ = base_node<S>((v[0] - o[0]) * ih[0], c.nx) - ox;
          const int ny_ = base_node<S>((v[2] - o[1]) * ih[1], c.ny) - oy;
          const int nz_ = base_node<S>((v[4] - o[2]) * ih[2], c.nz) - oz;
          stay = (unsigned)nx_ < (unsigned)sp.T[0] && (unsigned)ny_ < (unsigned)sp.T[1] &&
                 (unsigned)nz_ < (unsigned)sp.T[2];
        }
        const uint64_t m_s = __ballot(stay), m_m = __ballot(act && !stay);
        const int lane = (int)__lane_id();
        const uint64_t below = (1ull << lane) - 1ull;
        uint32_t b_s = 0u, b_m = 0u;
        if (lane == 0) {
          if (m_s) b_s = atomicAdd(&s_up, (uint32_t)__popcll(m_s));
          if (m_m) b_m = atomicSub(&s_down, (uint32_t)__popcll(m_m));
        }
        b_s = __shfl(b_s, 0);
        b_m = __shfl(b_m, 0);
        slot = stay ? (int64_t)b_s + __popcll(m_s & below)
                    : (int64_t)b_m - __popcll(m_m) + __popcll(m_m & below);
        if (act && (slot < ch.y || slot >= ch.z)) {  // impossible: the two ends tile the chunk
          bin_fault = true;
          slot = i;
        }
      }
      if (act) {
        for (int r = 0; r < 6; ++r) B[r * n + slot] = v[r];
        if constexpr (PERM)
          if (iddst) iddst[slot] = idsrc[i0];
      }
    }
  }
  if (bin_fault) atomicCAS(const_cast<int*>(&g->status), 0, -7);
  if (has_next) box_accumulate_block(lo, hi, bad, box);
  if constexpr (DIAG) {
    // wave sums, then the waves' sums through LDS (the window is free after the barrier; the
    // launch gives at least kMaxThreads / 64 * 27 doubles)
    for (int q = 0; q < kMomentSlots; ++q)
      for (int off = 32; off > 0; off >>= 1) acc[q] += __shfl_xor(acc[q], off);
    double* red = reinterpret_cast<double*>(smem_raw);
    const int wave = threadIdx.x >> 6, nwave = (int)(blockDim.x + 63) >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0)
      for (int q = 0; q < kMomentSlots; ++q) red[wave * kMomentSlots + q] = acc[q];
    __syncthreads();
    if (threadIdx.x < kMomentSlots) {
      double t = 0.0;
      for (int w = 0; w < nwave; ++w) t += red[w * kMomentSlots + threadIdx.x];
      diag_part[(int64_t)blk * kMomentSlots + threadIdx.x] = t;
    }
  }
}

// With DIAG the 27 moment sums stay in registers beside the particle's state: the kernel is
// built for at most kDiagThreads lanes per workgroup, which doubles the registers a lane may
// hold and keeps the sums out of scratch memory.
constexpr int kDiagThreads = 512;

template <int S, typename T, bool PERM, bool DIAG>
__global__ __launch_bounds__(DIAG ? kDiagThreads : kMaxThreads) void k_gkd_tiles(double* __restrict__ B,
                                                    const double* __restrict__ src,
                                                    const uint32_t* __restrict__ perm,
                                                    const uint32_t* __restrict__ idsrc,
                                                    uint32_t* __restrict__ iddst,
                                                    const Geom* __restrict__ g,
                                                    const T* __restrict__ E, Consts c,
                                                    SortPlan sp,
                                                    const int4* __restrict__ chunks,
                                                    const uint32_t* __restrict__ nchunks,
                                                    double L, HalfMap second, int has_next,
                                                    HalfMap first_next, Box* box,
                                                    double* __restrict__ diag_part,
                                                    const double* __restrict__ diag_shift) {
  gkd_tiles_body<S, T, PERM, DIAG>(B, src, perm, idsrc, iddst, g, E, c, sp, chunks, nchunks, L,
                                   second, has_next, first_next, box, blockIdx.x, gridDim.x,
                                   diag_part, diag_shift);
}

// The shift of the fused moment sums: the previous step's means (prev, 6 doubles), or, for the
// first step (prev == nullptr), the centre of the step's grid for the positions and 0 for the
// momenta.
__global__ void k_diag_shift(const Geom* __restrict__ g, Consts c, const double* __restrict__ prev,
                             double* __restrict__ shift) {
  const int r = threadIdx.x;
  if (r >= 6) return;
  if (prev) {
    shift[r] = prev[r];
  } else if (r & 1) {
    shift[r] = 0.0;
  } else {
    const int a = r >> 1;
    const int na = a == 0 ? c.nx : (a == 1 ? c.ny : c.nz);
    shift[r] = g->origin[a] + 0.5 * (na - 1) * g->h[a];
  }
}

// Moments from the blocks' partial sums: one wave per slot sums the nblk partials; then
// mean_r = shift_r + S_r / n and the centred products S_ab / n - (S_a / n)(S_b / n).  A device
// error state (status != 0) writes NaN.
__global__ __launch_bounds__(1024) void k_diag_combine(const Geom* __restrict__ g,
                                                       const double* __restrict__ part, int nblk,
                                                       const double* __restrict__ shift,
                                                       int64_t n, double* __restrict__ out) {
  __shared__ double tot[kMomentSlots];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, nwave = (int)blockDim.x >> 6;
  for (int q = wave; q < kMomentSlots; q += nwave) {
    double t = 0.0;
    for (int b = lane; b < nblk; b += 64) t += part[(int64_t)b * kMomentSlots + q];
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off);
    if (lane == 0) tot[q] = t;
  }
  __syncthreads();
  if (threadIdx.x >= kMomentSlots) return;
  const int q = threadIdx.x;
  if (g->status) {
    out[q] = NAN;
    return;
  }
  const double inv = 1.0 / (double)n;
  if (q < 6) {
    out[q] = shift[q] + tot[q] * inv;
    return;
  }
  int a = 0, k = q - 6;
  while (k >= 6 - a) {
    k -= 6 - a;
    ++a;
  }
  const int b = a + k;
  out[q] = tot[q] * inv - (tot[a] * inv) * (tot[b] * inv);
}

// First half of the first step out of the caller's array: A = drift(quad(X)), ids, box.  The
// ids are the caller's labels ids_in (binned order) or the indices in X; idA == nullptr: none.
__device__ __forceinline__ void prologue_body(const double* __restrict__ X,
                                                   double* __restrict__ A,
                                                   uint32_t* __restrict__ idA,
                                                   const uint32_t* __restrict__ ids_in,
                                                   const HalfMap& first, Consts c, Box* box,
                                                   int blk, int nblk) {
  const int64_t n = c.n;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  bool bad = false;
  for (int64_t i = blk * (int64_t)kBlk + threadIdx.x; i < n;
       i += (int64_t)nblk * kBlk) {
    double v[6];
    for (int r = 0; r < 6; ++r) v[r] = X[r * n + i];
    apply_half(first, v, c.inv_gamma2);
    for (int r = 0; r < 6; ++r) A[r * n + i] = v[r];
    if (idA) idA[i] = ids_in ? ids_in[i] : (uint32_t)i;
    double p[3] = {v[0], v[2], v[4]};
    for (int a = 0; a < 3; ++a) {
      bad |= !isfinite(p[a]);
      lo[a] = fmin(lo[a], p[a]);
      hi[a] = fmax(hi[a], p[a]);
    }
  }
  box_accumulate_block(lo, hi, bad, box);
}

__global__ __launch_bounds__(kBlk) void k_prologue(const double* __restrict__ X,
                                                   double* __restrict__ A,
                                                   uint32_t* __restrict__ idA,
                                                   const uint32_t* __restrict__ ids_in,
                                                   HalfMap first, Consts c, Box* box) {
  prologue_body(X, A, idA, ids_in, first, c, box, blockIdx.x, gridDim.x);
}

// Bucket keys for the return to the caller's order: key = id >> shift (at most 4096 buckets of
// consecutive original indices), with the block-privatised histogram of k_key_hist.
__device__ __forceinline__ void id_hist_body(const uint32_t* __restrict__ ids, int64_t n,
                                                  int shift, int nbuckets,
                                                  uint32_t* __restrict__ keys,
                                                  uint32_t* __restrict__ hist, int blk, int nblk) {
  __shared__ uint32_t lh[kMaxTiles];
  for (int t = threadIdx.x; t < nbuckets; t += kBlk) lh[t] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blk * kItems;
  for (int k = 0; k < kPer; ++k) {
    int64_t i = base + k * kBlk + threadIdx.x;
    if (i < n) {
      uint32_t key = ids[i] >> shift;
      key = key < (uint32_t)nbuckets ? key : (uint32_t)nbuckets - 1u;
      keys[i] = key;
      atomicAdd(&lh[key], 1u);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < nbuckets; t += kBlk)
    if (lh[t]) atomicAdd(&hist[t], lh[t]);
}

__global__ __launch_bounds__(kBlk) void k_id_hist(const uint32_t* __restrict__ ids, int64_t n,
                                                  int shift, int nbuckets,
                                                  uint32_t* __restrict__ keys,
                                                  uint32_t* __restrict__ hist) {
  id_hist_body(ids, n, shift, nbuckets, keys, hist, blockIdx.x, gridDim.x);
}

// Back to the caller's order: X[r][id[i]] = A[r][i].  After the bucket pass, the particles a
// block handles have ids in a narrow range, so its writes stay within an L2-sized window.
__device__ __forceinline__ void unpermute_body(const double* __restrict__ A,
                                                    const uint32_t* __restrict__ idA, int64_t n,
                                                    const Geom* __restrict__ g,
                                                    double* __restrict__ X, int blk, int nblk) {
  if (g->status) return;  // after a device error X keeps the caller's input
  for (int64_t i = blk * (int64_t)kBlk + threadIdx.x; i < n;
       i += (int64_t)nblk * kBlk) {
    uint32_t j = idA[i];
    if (j < (uint64_t)n)
      for (int r = 0; r < 6; ++r) X[r * n + j] = A[r * n + i];
  }
}

__global__ __launch_bounds__(kBlk) void k_unpermute(const double* __restrict__ A,
                                                    const uint32_t* __restrict__ idA, int64_t n,
                                                    const Geom* __restrict__ g,
                                                    double* __restrict__ X) {
  unpermute_body(A, idA, n, g, X, blockIdx.x, gridDim.x);
}


// Final placement through LDS.  After the bucket scatter, bucket b holds exactly the particles
// with ids [b 2^sh, (b + 1) 2^sh) (the ids are a permutation of 0..n-1), at those same
// positions of A.  One workgroup of kUBlk threads takes a bucket: each thread keeps the local
// offsets (id - b 2^sh) of its kUPer items; then, row by row, the values are dropped into an
// LDS buffer at their offsets, kUStage at a time, and written back to X contiguously, so every
// store is coalesced.  Each pass loads the row's items eight at a time (the second pass from
// L2) instead of holding all 32 in registers, which had spilled.  Requires 2^sh <= kUBlk *
// kUPer (= 32768).
constexpr int kUBlk = 1024;
constexpr int kUPer = 32;
constexpr int kUStage = 16384;

__global__ __launch_bounds__(kUBlk) void k_unpermute_lds(const double* __restrict__ A,
                                                         const uint32_t* __restrict__ idA,
                                                         int64_t n, int sh,
                                                         const Geom* __restrict__ g,
                                                         double* __restrict__ X) {
  __shared__ double stage[kUStage];
  if (g->status) return;  // after a device error X keeps the caller's input
  const int64_t b0 = (int64_t)blockIdx.x << sh;
  const int cnt = (int)min((int64_t)1 << sh, n - b0);
  // 16-bit offsets, two per register (2^sh <= 32768); 0xffff marks no item.  An id outside
  // the bucket (impossible for a permutation) is dropped, so LDS stays in bounds.
  uint32_t offp[kUPer / 2];
#pragma unroll
  for (int k = 0; k < kUPer; ++k) {
    const int l = threadIdx.x + k * kUBlk;
    uint32_t o = 0xffffu;
    if (l < cnt) {
      const int64_t d = (int64_t)idA[b0 + l] - b0;
      if (d >= 0 && d < cnt) o = (uint32_t)d;
    }
    if (k & 1)
      offp[k >> 1] |= o << 16;
    else
      offp[k >> 1] = o;
  }
  const int nq = (cnt + kUStage - 1) / kUStage;
  for (int r = 0; r < 6; ++r) {
    for (int q = 0; q < nq; ++q) {
      // eight loads in flight per thread, unconditional (clamped into the bucket, cnt >= 1),
      // then the stores of the items whose offset falls in this pass
#pragma unroll 1
      for (int k0 = 0; k0 < kUPer; k0 += 8) {
        double v[8];
#pragma unroll
        for (int j = 0; j < 8; ++j)
          v[j] = A[r * n + b0 + min((int)threadIdx.x + (k0 + j) * kUBlk, cnt - 1)];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int k = k0 + j;
          const uint32_t o = (offp[k >> 1] >> (16 * (k & 1))) & 0xffffu;
          if (o != 0xffffu && (int)(o / kUStage) == q) stage[o % kUStage] = v[j];
        }
      }
      __syncthreads();
      const int len = min(kUStage, cnt - q * kUStage);
      for (int t = threadIdx.x; t < len; t += kUBlk) X[r * n + b0 + q * kUStage + t] = stage[t];
      __syncthreads();
    }
  }
}

// ------------------------------------------------------------------------ batched wrappers
// beam = blockIdx.y; the current phase-space copy of step j is XA for even j (parity 0).

__device__ __forceinline__ double* cur_X(const BeamDev& d, int parity) { return parity ? d.XB : d.XA; }
__device__ __forceinline__ double* nxt_X(const BeamDev& d, int parity) { return parity ? d.XA : d.XB; }
__device__ __forceinline__ uint32_t* cur_id(const BeamDev& d, int parity) { return parity ? d.idB : d.idA; }
__device__ __forceinline__ uint32_t* nxt_id(const BeamDev& d, int parity) { return parity ? d.idA : d.idB; }

__global__ __launch_bounds__(kBlk) void k_prologue_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  prologue_body(d.X, d.XA, d.idA, nullptr, d.slices[0].first, d.c, d.box, blockIdx.x, gridDim.x);
}

template <int S>
__global__ __launch_bounds__(kBlk) void k_key_hist_batch(const BeamDev* __restrict__ beams,
                                                         int parity) {
  const BeamDev& d = beams[blockIdx.y];
  if ((int64_t)blockIdx.x * kItems >= d.c.n) return;
  key_hist_body<S>(cur_X(d, parity), d.geom, d.c, d.sp, d.keys, d.hist, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(1024) void k_build_chunks_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.x];
  build_chunks_body(d.geom, d.sp, d.hist, d.cursor, d.chunks, d.nchunks);
}

// after a call's first step: the ranking only (cur_X stays where it is)
__global__ __launch_bounds__(kBlk) void k_scatter_perm_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  if ((int64_t)blockIdx.x * kItems >= d.c.n) return;
  scatter_perm_body(d.keys, d.geom, d.c.n, d.sp.ntiles, d.cursor, d.perm, blockIdx.x);
}

template <bool STAGED>
__global__ __launch_bounds__(kBlk) void k_scatter_batch(const BeamDev* __restrict__ beams,
                                                        int parity) {
  const BeamDev& d = beams[blockIdx.y];
  if ((int64_t)blockIdx.x * kItems >= d.c.n) return;
  scatter_body<STAGED>(cur_X(d, parity), cur_id(d, parity), d.keys, d.geom, d.c.n, d.sp.ntiles, d.cursor,
               nxt_X(d, parity), nxt_id(d, parity), blockIdx.x, gridDim.x);
}

// PERM: the step's input cur_X through the ranking; else nxt_X, in slot order
template <int S, typename T, bool PERM>
__global__ __launch_bounds__(kBlk) void k_deposit_tiles_batch(const BeamDev* __restrict__ beams,
                                                              int parity) {
  const BeamDev& d = beams[blockIdx.y];
  deposit_tiles_body<S, T, PERM>(PERM ? cur_X(d, parity) : nxt_X(d, parity),
                                 PERM ? d.perm : nullptr, d.geom, d.c, d.sp, d.chunks,
                                 d.nchunks, (T*)d.rho, blockIdx.x, gridDim.x, d.tacc, d.tscale);
}

template <int S, typename T>
__global__ __launch_bounds__(256) void k_tile_reduce_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  tile_reduce_body<S, T>(d.geom, d.c, d.sp, d.tacc, d.tscale, (T*)d.rho, blockIdx.x, gridDim.x);
}

// every beam's per-tile integer windows set to zero (once per batch call)
__global__ __launch_bounds__(256) void k_clear_tacc_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.y];
  const int S = d.c.shape;
  const int64_t count = (int64_t)d.sp.ntiles * (d.sp.T[0] + S) * (d.sp.T[1] + S) * (d.sp.T[2] + S);
  for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < count; i += (int64_t)gridDim.x * 256)
    d.tacc[i] = 0ull;
}

// PERM: reads cur_X (and its ids) through the ranking and writes nxt_X in slot order; else
// updates nxt_X in place
template <int S, typename T, bool PERM>
__global__ __launch_bounds__(kBlk) void k_gkd_tiles_batch(const BeamDev* __restrict__ beams,
                                                          int parity, int j, int n_steps) {
  const BeamDev& d = beams[blockIdx.y];
  const SliceDev& sl = d.slices[j % d.n_slices];
  const SliceDev& sn = d.slices[(j + 1) % d.n_slices];
  gkd_tiles_body<S, T, PERM, false>(nxt_X(d, parity), PERM ? cur_X(d, parity) : nullptr,
                                    PERM ? d.perm : nullptr, PERM ? cur_id(d, parity) : nullptr,
                                    PERM ? nxt_id(d, parity) : nullptr, d.geom, (const T*)d.E,
                                    d.c, d.sp, d.chunks, d.nchunks, sl.L, sl.second,
                                    j + 1 < n_steps, sn.first, d.box, blockIdx.x, gridDim.x);
}

// reordering at the end: bucket keys of the ids, bucket offsets, bucket scatter, final scatter
__device__ __forceinline__ void bucket_plan(int64_t n, int* shift, int* nb) {
  int sh = 0;
  while (((n - 1) >> sh) >= kMaxTiles) ++sh;
  *shift = sh;
  *nb = (int)(((n - 1) >> sh) + 1);
}

__global__ __launch_bounds__(kBlk) void k_id_hist_batch(const BeamDev* __restrict__ beams,
                                                        int parity) {
  const BeamDev& d = beams[blockIdx.y];
  if ((int64_t)blockIdx.x * kItems >= d.c.n) return;
  int sh, nb;
  bucket_plan(d.c.n, &sh, &nb);
  id_hist_body(cur_id(d, parity), d.c.n, sh, nb, d.keys, d.hist, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(1024) void k_bucket_chunks_batch(const BeamDev* __restrict__ beams) {
  const BeamDev& d = beams[blockIdx.x];
  int sh, nb;
  bucket_plan(d.c.n, &sh, &nb);
  SortPlan bp;
  bp.T[0] = bp.T[1] = bp.T[2] = 1;
  bp.NT[0] = nb;
  bp.NT[1] = bp.NT[2] = 1;
  bp.ntiles = nb;
  bp.chunk = 1 << 30;
  bp.max_chunks = nb + 1;
  build_chunks_body(d.geom, bp, d.hist, d.cursor, d.chunks, d.nchunks);
}

__global__ __launch_bounds__(kBlk) void k_bucket_scatter_batch(const BeamDev* __restrict__ beams,
                                                               int parity) {
  const BeamDev& d = beams[blockIdx.y];
  if ((int64_t)blockIdx.x * kItems >= d.c.n) return;
  int sh, nb;
  bucket_plan(d.c.n, &sh, &nb);
  scatter_body<true>(cur_X(d, parity), cur_id(d, parity), d.keys, d.geom, d.c.n, nb, d.cursor,
               nxt_X(d, parity), nxt_id(d, parity), blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(kBlk) void k_unpermute_batch(const BeamDev* __restrict__ beams,
                                                          int parity) {
  const BeamDev& d = beams[blockIdx.y];
  unpermute_body(nxt_X(d, parity), nxt_id(d, parity), d.c.n, d.geom, d.X, blockIdx.x, gridDim.x);
}

int grid_items(int64_t n) { return (int)((n + kItems - 1) / kItems); }
int grid_wide(int64_t n) { return (int)((n + kWItems - 1) / kWItems); }
// the wide staged scatter once it still fills every CU with a block (256 CUs); below that the
// 4096-particle blocks of k_scatter<true> keep the device busy
bool wide_pays(int64_t n) { return grid_wide(n) >= 256; }

int grid_stride(int64_t n) {
  int64_t b = (n + kBlk - 1) / kBlk;
  if (b > 8192) b = 8192;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

SortPlan make_sort_plan(int nx, int ny, int nz, int64_t n, const int tile[3], int chunk,
                        int blocks, int threads, int deposit_threads) {
  SortPlan sp;
  int nn[3] = {nx, ny, nz};
  for (int a = 0; a < 3; ++a) {
    int t = (nn[a] + 15) / 16;
    if (t < 4) t = 4;
    sp.T[a] = tile && tile[a] > 0 ? tile[a] : t;
    sp.NT[a] = (nn[a] + sp.T[a] - 1) / sp.T[a];
  }
  sp.ntiles = sp.NT[0] * sp.NT[1] * sp.NT[2];
  sp.chunk = chunk > 0 ? chunk : 8192;
  // every tile adds at most one partial work item
  const int64_t items = (int64_t)(n / sp.chunk) + sp.ntiles + 1;
  sp.max_chunks = items;
  // the work list also serves the id buckets of the final reordering (up to kMaxTiles entries)
  if (sp.max_chunks < kMaxTiles + 1) sp.max_chunks = kMaxTiles + 1;
  sp.blocks = blocks > 0 ? blocks : (int)(items < 4096 ? items : 4096);
  sp.threads = threads > 0 ? threads : kBlk;
  sp.dep_threads = deposit_threads > 0 ? deposit_threads : sp.threads;
  return sp;
}

namespace {
// Dynamic LDS above 64 KB needs the kernel's limit raised first; the runtime accepts a limit up
// to the device's 160 KB less the kernel's static LDS.
template <typename K>
hipError_t lds_optin(K kernel, size_t bytes) {
  if (bytes > kMaxLdsBytes) return hipErrorInvalidConfiguration;
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}
}  // namespace

#define PIC_TRY_LDS(kernel, bytes)            \
  do {                                        \
    hipError_t e_ = lds_optin(kernel, bytes); \
    if (e_ != hipSuccess) return e_;          \
  } while (0)

hipError_t launch_prologue(const double* X, double* A, uint32_t* idA, const uint32_t* ids_in,
                           const HalfMap& first, Consts c, Box* box, hipStream_t s) {
  hipLaunchKernelGGL(k_prologue, dim3(grid_stride(c.n)), dim3(kBlk), 0, s, X, A, idA, ids_in,
                     first, c, box);
  return hipGetLastError();
}

namespace {
// tile keys, histogram, sort offsets and the deposit work list of the particles in A
hipError_t launch_keys_chunks(const double* A, const Geom* g, Consts c, const SortPlan& sp,
                              uint32_t* keys, uint32_t* hist, uint32_t* cursor, int4* chunks,
                              uint32_t* nchunks, hipStream_t s) {
  if (c.shape == 1)
    hipLaunchKernelGGL(k_key_hist<1>, dim3(grid_items(c.n)), dim3(kBlk), 0, s, A, g, c, sp, keys,
                       hist);
  else
    hipLaunchKernelGGL(k_key_hist<2>, dim3(grid_items(c.n)), dim3(kBlk), 0, s, A, g, c, sp, keys,
                       hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_build_chunks, dim3(1), dim3(1024), 0, s, g, sp, hist, cursor, chunks,
                     nchunks);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_bin(const double* A, const uint32_t* idA, const Geom* g, Consts c,
                      const SortPlan& sp, uint32_t* keys, uint32_t* hist, uint32_t* cursor,
                      int4* chunks, uint32_t* nchunks, double* B, uint32_t* idB, bool staged,
                      hipStream_t s) {
  hipError_t e = launch_keys_chunks(A, g, c, sp, keys, hist, cursor, chunks, nchunks, s);
  if (e != hipSuccess) return e;
  if (staged && wide_pays(c.n))
    hipLaunchKernelGGL(k_scatter_wide, dim3(grid_wide(c.n)), dim3(kWBlk), 0, s, A, idA, keys, g,
                       c.n, sp.ntiles, cursor, B, idB);
  else if (staged)
    hipLaunchKernelGGL(k_scatter<true>, dim3(grid_items(c.n)), dim3(kBlk), 0, s, A, idA, keys, g,
                       c.n, sp.ntiles, cursor, B, idB);
  else
    hipLaunchKernelGGL(k_scatter<false>, dim3(grid_items(c.n)), dim3(kBlk), 0, s, A, idA, keys, g,
                       c.n, sp.ntiles, cursor, B, idB);
  return hipGetLastError();
}

hipError_t launch_bin_perm(const double* A, const Geom* g, Consts c, const SortPlan& sp,
                           uint32_t* keys, uint32_t* hist, uint32_t* cursor, int4* chunks,
                           uint32_t* nchunks, uint32_t* perm, hipStream_t s) {
  hipError_t e = launch_keys_chunks(A, g, c, sp, keys, hist, cursor, chunks, nchunks, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_perm, dim3(grid_items(c.n)), dim3(kBlk), 0, s, keys, g, c.n,
                     sp.ntiles, cursor, perm);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_deposit_tiles(const double* B, const uint32_t* perm, const Geom* g, Consts c,
                                const SortPlan& sp, const int4* chunks, const uint32_t* nchunks,
                                T* rho, hipStream_t s, unsigned long long* tacc, int* tscale) {
  const int S = c.shape;
  size_t lds = sizeof(unsigned long long) * (size_t)(sp.T[0] + S) * (sp.T[1] + S) * (sp.T[2] + S);
  const dim3 grid((unsigned)sp.blocks), block((unsigned)sp.dep_threads);
  if (!tacc || !tscale) return hipErrorInvalidValue;
  const int64_t nodes = (int64_t)c.nx * c.ny * c.nz;
  int rb = (int)((nodes + 255) / 256);
  if (rb > 16384) rb = 16384;
  if (S == 1) {
    PIC_TRY_LDS((k_deposit_tiles<1, T>), lds);
    hipLaunchKernelGGL((k_deposit_tiles<1, T>), grid, block, lds, s, B, perm, g, c, sp, chunks,
                       nchunks, rho, tacc, tscale);
    PIC_TRY(hipGetLastError());
    if (tacc)
      hipLaunchKernelGGL((k_tile_reduce<1, T>), dim3(rb), dim3(256), 0, s, g, c, sp, tacc, tscale,
                         rho);
  } else {
    PIC_TRY_LDS((k_deposit_tiles<2, T>), lds);
    hipLaunchKernelGGL((k_deposit_tiles<2, T>), grid, block, lds, s, B, perm, g, c, sp, chunks,
                       nchunks, rho, tacc, tscale);
    PIC_TRY(hipGetLastError());
    if (tacc)
      hipLaunchKernelGGL((k_tile_reduce<2, T>), dim3(rb), dim3(256), 0, s, g, c, sp, tacc, tscale,
                         rho);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_vdeposit_tiles(const double* B, const Geom* g, Consts c, const SortPlan& sp,
                                 const int4* chunks, const uint32_t* nchunks, T* e,
                                 hipStream_t s) {
  const int S = c.shape;
  const size_t lds = 3 * sizeof(double) * (size_t)(sp.T[0] + S) * (sp.T[1] + S) * (sp.T[2] + S);
  const dim3 grid((unsigned)sp.blocks), block((unsigned)sp.threads);
  if (S == 1) {
    PIC_TRY_LDS((k_vdeposit_tiles<1, T>), lds);
    hipLaunchKernelGGL((k_vdeposit_tiles<1, T>), grid, block, lds, s, B, g, c, sp, chunks, nchunks,
                       e);
  } else {
    PIC_TRY_LDS((k_vdeposit_tiles<2, T>), lds);
    hipLaunchKernelGGL((k_vdeposit_tiles<2, T>), grid, block, lds, s, B, g, c, sp, chunks, nchunks,
                       e);
  }
  return hipGetLastError();
}

template hipError_t launch_vdeposit_tiles<double>(const double*, const Geom*, Consts,
                                                  const SortPlan&, const int4*, const uint32_t*,
                                                  double*, hipStream_t);
template hipError_t launch_vdeposit_tiles<float>(const double*, const Geom*, Consts,
                                                 const SortPlan&, const int4*, const uint32_t*,
                                                 float*, hipStream_t);

template <typename T>
hipError_t launch_gkd_tiles(double* B, const double* src, const uint32_t* perm,
                            const uint32_t* idsrc, uint32_t* iddst, const Geom* g, const T* E,
                            Consts c, const SortPlan& sp, const int4* chunks,
                            const uint32_t* nchunks, double L, const HalfMap& second,
                            int has_next, const HalfMap& first_next, Box* box, hipStream_t s,
                            double* diag_part, double* diag_shift, const double* diag_prev,
                            double* diag_out) {
  const int S = c.shape;
  size_t lds = 3 * sizeof(T) * (size_t)(sp.T[0] + S) * (sp.T[1] + S) * (sp.T[2] + S);
  const bool diag = diag_out != nullptr;
  const dim3 grid((unsigned)sp.blocks),
      block((unsigned)(diag ? std::min(sp.threads, kDiagThreads) : sp.threads));
  // the ids are optional, as a pair
  if (perm && (!src || src == B || (!idsrc != !iddst) || (idsrc && idsrc == iddst)))
    return hipErrorInvalidValue;
  if (diag) {
    if (!diag_part || !diag_shift) return hipErrorInvalidValue;
    const size_t red = sizeof(double) * kMomentSlots * (kMaxThreads / 64);
    if (lds < red) lds = red;
    hipLaunchKernelGGL(k_diag_shift, dim3(1), dim3(64), 0, s, g, c, diag_prev, diag_shift);
    PIC_TRY(hipGetLastError());
  }
#define PIC_GKD(SS, PP, DD)                                                                   \
  do {                                                                                        \
    PIC_TRY_LDS((k_gkd_tiles<SS, T, PP, DD>), lds);                                           \
    hipLaunchKernelGGL((k_gkd_tiles<SS, T, PP, DD>), grid, block, lds, s, B, src, perm, idsrc,\
                       iddst, g, E, c, sp, chunks, nchunks, L, second, has_next, first_next,  \
                       box, diag_part, diag_shift);                                           \
  } while (0)
  if (diag) {
    if (S == 1) {
      if (perm) PIC_GKD(1, true, true); else PIC_GKD(1, false, true);
    } else {
      if (perm) PIC_GKD(2, true, true); else PIC_GKD(2, false, true);
    }
  } else {
    if (S == 1) {
      if (perm) PIC_GKD(1, true, false); else PIC_GKD(1, false, false);
    } else {
      if (perm) PIC_GKD(2, true, false); else PIC_GKD(2, false, false);
    }
  }
#undef PIC_GKD
  PIC_TRY(hipGetLastError());
  if (diag) {
    hipLaunchKernelGGL(k_diag_combine, dim3(1), dim3(1024), 0, s, g, diag_part, sp.blocks,
                       diag_shift, c.n, diag_out);
    PIC_TRY(hipGetLastError());
  }
  return hipSuccess;
}

template hipError_t launch_gkd_tiles<double>(double*, const double*, const uint32_t*,
                                             const uint32_t*, uint32_t*, const Geom*,
                                             const double*, Consts, const SortPlan&, const int4*,
                                             const uint32_t*, double, const HalfMap&, int,
                                             const HalfMap&, Box*, hipStream_t, double*, double*,
                                             const double*, double*);
template hipError_t launch_gkd_tiles<float>(double*, const double*, const uint32_t*,
                                            const uint32_t*, uint32_t*, const Geom*, const float*,
                                            Consts, const SortPlan&, const int4*, const uint32_t*,
                                            double, const HalfMap&, int, const HalfMap&, Box*,
                                            hipStream_t, double*, double*, const double*,
                                            double*);

hipError_t launch_unpermute(const double* A, const uint32_t* idA, int64_t n, double* X,
                            uint32_t* keys, uint32_t* hist, uint32_t* cursor, int4* chunks,
                            uint32_t* nchunks, double* B, uint32_t* idB, const Geom* g,
                            hipStream_t s) {
  int shift = 0;
  while (((n - 1) >> shift) >= kMaxTiles) ++shift;
  const int nb = (int)(((n - 1) >> shift) + 1);
  SortPlan bp;
  bp.T[0] = bp.T[1] = bp.T[2] = 1;
  bp.NT[0] = nb;
  bp.NT[1] = bp.NT[2] = 1;
  bp.ntiles = nb;
  bp.chunk = 1 << 30;  // the work list is not used; one entry per bucket
  bp.max_chunks = nb + 1;
  hipLaunchKernelGGL(k_id_hist, dim3(grid_items(n)), dim3(kBlk), 0, s, idA, n, shift, nb, keys,
                     hist);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_build_chunks, dim3(1), dim3(1024), 0, s, g, bp, hist, cursor, chunks,
                     nchunks);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (wide_pays(n))
    hipLaunchKernelGGL(k_scatter_wide, dim3(grid_wide(n)), dim3(kWBlk), 0, s, A, idA, keys, g, n,
                       nb, cursor, B, idB);
  else
    hipLaunchKernelGGL(k_scatter<true>, dim3(grid_items(n)), dim3(kBlk), 0, s, A, idA, keys, g, n,
                       nb, cursor, B, idB);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (((int64_t)1 << shift) <= (int64_t)kUBlk * kUPer)
    hipLaunchKernelGGL(k_unpermute_lds, dim3(nb), dim3(kUBlk), 0, s, B, idB, n, shift, g, X);
  else
    hipLaunchKernelGGL(k_unpermute, dim3(grid_stride(n)), dim3(kBlk), 0, s, B, idB, n, g, X);
  return hipGetLastError();
}

// ------------------------------------------------------------------------ batched launches

hipError_t launch_batch_prologue_particles(const BeamDev* beams, int nb, const BatchDims& bd,
                                           hipStream_t s) {
  hipLaunchKernelGGL(k_prologue_batch, dim3(grid_stride(bd.max_n), nb), dim3(kBlk), 0, s, beams);
  return hipGetLastError();
}

hipError_t launch_batch_particles_bin(const BeamDev* beams, int nb, const BatchDims& bd, int shape,
                                      int parity, bool first, hipStream_t s) {
  const dim3 grid(grid_items(bd.max_n), nb);
  if (shape == 1)
    hipLaunchKernelGGL(k_key_hist_batch<1>, grid, dim3(kBlk), 0, s, beams, parity);
  else
    hipLaunchKernelGGL(k_key_hist_batch<2>, grid, dim3(kBlk), 0, s, beams, parity);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_build_chunks_batch, dim3(nb), dim3(1024), 0, s, beams);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the first step moves the caller's order into tile order (staged scatter); later steps, whose
  // input is in the previous step's tile order, only rank
  if (first)
    hipLaunchKernelGGL(k_scatter_batch<true>, grid, dim3(kBlk), 0, s, beams, parity);
  else
    hipLaunchKernelGGL(k_scatter_perm_batch, grid, dim3(kBlk), 0, s, beams);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_deposit(const BeamDev* beams, int nb, const BatchDims& bd, int shape,
                                int parity, bool first, hipStream_t s) {
  const dim3 grid(bd.max_chunks, nb);
  int rb = (int)(((int64_t)bd.max_nx * bd.max_ny * bd.max_nz + 255) / 256);
  if (rb > 16384) rb = 16384;
#define PIC_DEP_BATCH(SS, PP)                                                                 \
  do {                                                                                        \
    PIC_TRY_LDS((k_deposit_tiles_batch<SS, T, PP>), bd.dep_lds);                              \
    hipLaunchKernelGGL((k_deposit_tiles_batch<SS, T, PP>), grid, dim3(kBlk), bd.dep_lds, s,   \
                       beams, parity);                                                        \
    PIC_TRY(hipGetLastError());                                                               \
    hipLaunchKernelGGL((k_tile_reduce_batch<SS, T>), dim3(rb, nb), dim3(256), 0, s, beams);   \
  } while (0)
  if (shape == 1) {
    if (first) PIC_DEP_BATCH(1, false); else PIC_DEP_BATCH(1, true);
  } else {
    if (first) PIC_DEP_BATCH(2, false); else PIC_DEP_BATCH(2, true);
  }
#undef PIC_DEP_BATCH
  return hipGetLastError();
}

hipError_t launch_batch_clear_tacc(const BeamDev* beams, int nb, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_tacc_batch, dim3(1024, nb), dim3(256), 0, s, beams);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_batch_gkd(const BeamDev* beams, int nb, const BatchDims& bd, int shape,
                            int parity, int j, int n_steps, bool first, hipStream_t s) {
  const dim3 grid(bd.max_chunks, nb);
#define PIC_GKD_BATCH(SS, PP)                                                                 \
  do {                                                                                        \
    PIC_TRY_LDS((k_gkd_tiles_batch<SS, T, PP>), bd.gkd_lds);                                  \
    hipLaunchKernelGGL((k_gkd_tiles_batch<SS, T, PP>), grid, dim3(kBlk), bd.gkd_lds, s, beams, \
                       parity, j, n_steps);                                                   \
  } while (0)
  if (shape == 1) {
    if (first) PIC_GKD_BATCH(1, false); else PIC_GKD_BATCH(1, true);
  } else {
    if (first) PIC_GKD_BATCH(2, false); else PIC_GKD_BATCH(2, true);
  }
#undef PIC_GKD_BATCH
  return hipGetLastError();
}

hipError_t launch_batch_unpermute(const BeamDev* beams, int nb, const BatchDims& bd, int parity,
                                  hipStream_t s) {
  const dim3 grid(grid_items(bd.max_n), nb);
  hipLaunchKernelGGL(k_id_hist_batch, grid, dim3(kBlk), 0, s, beams, parity);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bucket_chunks_batch, dim3(nb), dim3(1024), 0, s, beams);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bucket_scatter_batch, grid, dim3(kBlk), 0, s, beams, parity);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_unpermute_batch, dim3(grid_stride(bd.max_n), nb), dim3(kBlk), 0, s, beams,
                     parity);
  return hipGetLastError();
}

template hipError_t launch_batch_deposit<double>(const BeamDev*, int, const BatchDims&, int, int,
                                                 bool, hipStream_t);
template hipError_t launch_batch_deposit<float>(const BeamDev*, int, const BatchDims&, int, int,
                                                bool, hipStream_t);
template hipError_t launch_batch_gkd<double>(const BeamDev*, int, const BatchDims&, int, int, int,
                                             int, bool, hipStream_t);
template hipError_t launch_batch_gkd<float>(const BeamDev*, int, const BatchDims&, int, int, int,
                                            int, bool, hipStream_t);

template hipError_t launch_deposit_tiles<double>(const double*, const uint32_t*, const Geom*,
                                                 Consts, const SortPlan&, const int4*,
                                                 const uint32_t*, double*, hipStream_t,
                                                 unsigned long long*, int*);
template hipError_t launch_deposit_tiles<float>(const double*, const uint32_t*, const Geom*,
                                                Consts, const SortPlan&, const int4*,
                                                const uint32_t*, float*, hipStream_t,
                                                unsigned long long*, int*);

}  // namespace pic
