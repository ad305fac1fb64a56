// One query spread over the whole device: sDTW (Eq. 1, int16 path) as M
// row-wide scans with a decoupled look-back between column tiles.
//
// Along a row the recurrence is a linear one in the (min, +) semiring.  With
// d_j = |x_i - y_j| and a_j = d_j + min(gamma(i-1, j-1), gamma(i-1, j)),
//   gamma(i, j) = min(a_j, gamma(i, j-1) + d_j),
// i.e. gamma(i, j) = f_j(gamma(i, j-1)) for the map f_j(x) = min(a_j, x + d_j).
// Maps of the form x -> min(A, x + D) are closed under composition (f then g
// is (min(A_g, A_f + D_g), D_f + D_g)), so a row is a prefix scan of maps
// applied to gamma(i, 0) = +inf: a row's cells no longer wait for their left
// neighbour one by one, and the N columns of a row are computed by every
// compute unit at once.  Integer costs make the reassociated sums exact, so
// results equal the cell-by-cell recurrence bit for bit.
//
// One workgroup of 256 threads per tile of 256 C columns (thread t owns C
// consecutive columns; its previous row stays in registers).  Per row:
//   1. every thread composes the maps of its C cells;
//   2. a workgroup scan gives each thread the map of the columns left of it
//      within the tile, and the tile's map;
//   3. the tile publishes its map, then its first wave looks back over the
//      flags of the tiles to its left (64 at a time, then over the maps of
//      whole groups of 64 tiles), composing maps until it meets a tile that
//      has published its last value of the row, which gives
//      gamma(i, first column - 1); the tile publishes its own last value;
//   4. every thread applies its map prefix to that value and sweeps its C
//      cells again, producing the row.
// Extending a resident row (a stream: the row gamma(m_old, .) of the rows
// folded in so far), the tile starts from that row instead of the free-start
// zeros and writes its last row back over it.  A tile's first thread needs
// the old value left of the tile, which the tile to its left may already
// have overwritten (tiles beyond those resident run later), so the clearing
// kernel takes a copy of every tile's left neighbour value first.
// Tiles take their index from an atomic ticket, so a tile waits only on
// tiles that started before it; a tile that waits far too long (about a
// second; only a defect could cause it) raises an abort flag that ends every
// wait, and the launch then reports -1 for cost and end.
//
// Value ranges (32-bit): costs < 2^28 (M <= 4096 rows of |x - y| <= 65535),
// +inf = 2^31, a tile's D < 2^30 (at most 16,384 columns), and the look-back
// saturates the D it accumulates at 2^30 - 1, the largest value the 30-bit D
// field of a flag word holds: x + D then still exceeds every cost, so the
// min picks the same value as with the exact sum, and kInf + D < 2^32.
#include <limits.h>

#include <mutex>

#include "common.h"

namespace sdtw {

// Scratch of sdtw_align_one_wide_noalloc: one fixed array per device (every
// device the library runs on holds it until the process ends), so that the
// call allocates nothing.  Host code never passes the array's name to a
// kernel (on the host it is a stand-in, not a device address); it passes the
// address hipGetSymbolAddress returns for the current device.
constexpr int64_t kNoallocWords = int64_t(1) << 20;  // 64-bit words: 8 MiB
static __device__ __align__(256) uint64_t g_noalloc_scratch[kNoallocWords];

namespace {

constexpr int kWideThreads = 256;
constexpr int kLookback = 64;  // tiles one look-back round trip covers (one per lane)
constexpr uint32_t kInf = 1u << 31;
constexpr uint32_t kDCap = (1u << 30) - 1;  // largest D a flag word's 30-bit field holds
constexpr uint64_t kAgg = 1, kIncl = 2;  // flag status, low two bits of a flag word
constexpr uint32_t kSpinLimit = 1u << 20;  // polling rounds (each a memory round trip) before
                                           // a wait aborts: about a second

struct Map {
  uint32_t a, d;  // x -> min(a, x + d)
};

__device__ __forceinline__ Map compose(Map f, Map g) {  // f, then g
  Map r;
  r.a = min(g.a, f.a + g.d);
  r.d = f.d + g.d;
  return r;
}

// Composition that saturates D at kDCap (both inputs <= kDCap): used where
// many tiles' maps are combined.
__device__ __forceinline__ Map compose_sat(Map f, Map g) {
  Map r;
  r.a = min(g.a, f.a + g.d);
  r.d = min(f.d + g.d, kDCap);
  return r;
}

// |x - y| + acc, and a_j = |x - y_j| + min(gamma(i-1, j-1), gamma(i-1, j)).
// Plain code lets the compiler keep each cell's distance and a_j from the
// first sweep for the second (fewer instructions, a shorter row); the
// LowReg forms are asm, so the second sweep recomputes them and a thread
// needs about 2C registers instead of 3-4C, which fits more tiles on the
// device at once (worth it only when the tiles would otherwise run in more
// rounds).
template <bool LowReg>
__device__ __forceinline__ uint32_t sad(uint32_t x, uint32_t y, uint32_t acc) {
  if constexpr (LowReg) {
    uint32_t r;
    asm volatile("v_sad_u32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(y), "v"(acc));
    return r;
  } else {
    return (x > y ? x - y : y - x) + acc;
  }
}
template <bool LowReg>
__device__ __forceinline__ uint32_t cell_a(uint32_t x, uint32_t y, uint32_t diag, uint32_t up) {
  if constexpr (LowReg) {
    uint32_t m;
    asm volatile("v_min_u32 %0, %1, %2" : "=v"(m) : "v"(diag), "v"(up));
    return sad<true>(x, y, m);
  } else {
    return sad<false>(x, y, min(diag, up));
  }
}

// A flag word carries its payload (a map or a value) with its status in one
// 64-bit word, so readers need no ordering with other memory: relaxed
// device-scope atomics suffice (coherent across the XCDs' L2s), and no
// release or acquire fence writes back or invalidates the L2 on every
// publish and poll.
__device__ __forceinline__ uint64_t load_flag(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_flag(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup exclusive scan of maps in thread order; also the total.
__device__ __forceinline__ Map scan_maps(Map m, Map& total, uint32_t* sa, uint32_t* sd) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  Map inc = m;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    Map o;
    o.a = (uint32_t)__shfl_up((int)inc.a, off);
    o.d = (uint32_t)__shfl_up((int)inc.d, off);
    if (lane >= off) inc = compose(o, inc);
  }
  if (lane == 63) {
    sa[wave] = inc.a;
    sd[wave] = inc.d;
  }
  Map ex;
  ex.a = (uint32_t)__shfl_up((int)inc.a, 1);
  ex.d = (uint32_t)__shfl_up((int)inc.d, 1);
  if (lane == 0) ex = Map{kInf, 0};
  __syncthreads();
  Map before{kInf, 0};
  total = Map{kInf, 0};
#pragma unroll
  for (int w = 0; w < kWideThreads / 64; ++w) {
    const Map t{sa[w], sd[w]};
    if (w < wave) before = compose(before, t);
    total = compose(total, t);
  }
  return compose(before, ex);
}

__device__ __forceinline__ uint64_t pack_agg(Map f) {
  return ((uint64_t)f.a << 32) | ((uint64_t)f.d << 2) | kAgg;
}
__device__ __forceinline__ Map unpack_agg(uint64_t w) {
  return Map{(uint32_t)(w >> 32), (uint32_t)(w & 0xFFFFFFFFu) >> 2};
}

// Composition of the maps of lanes 0 .. 63 (lane 0 nearest, so higher lanes
// are applied first), in every lane.
__device__ __forceinline__ Map wave_compose(Map f) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    Map o;
    o.a = (uint32_t)__shfl_down((int)f.a, off);
    o.d = (uint32_t)__shfl_down((int)f.d, off);
    if (lane + off < 64) f = compose_sat(o, f);
  }
  Map r;
  r.a = (uint32_t)__shfl((int)f.a, 0);
  r.d = (uint32_t)__shfl((int)f.d, 0);
  return r;
}

// One polling round found a flag missing: false to poll again, true when the
// launch is to give up (this wait took too long, or another one did).
__device__ __forceinline__ bool give_up(uint32_t& spins, uint32_t* ctrl) {
  bool stop = ++spins > kSpinLimit;
  stop = stop || __hip_atomic_load(&ctrl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
  if (__ballot(stop)) {  // uniform over the wave
    if ((threadIdx.x & 63) == 0)
      __hip_atomic_store(&ctrl[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return true;
  }
  __builtin_amdgcn_s_sleep(1);
  return false;
}

// gamma(i, first column of `tile` - 1), by wave 0 of the tile.  Flag words,
// per row i: agg[t] (the tile's map), inc[t] (gamma at its last column) and,
// per group of 64 tiles, gag[g] (the group's map, published by its last
// tile).  Two levels, so that a row costs a few memory round trips however
// many tiles there are:
//   1. the tiles of this tile's group to its left (one window): the nearest
//      one with inc published gives the value, composed with the maps of the
//      tiles in between; the group's last tile composes all of them into gag;
//   2. otherwise, with the maps of all those tiles composed, the groups to
//      the left, 64 per window: the nearest group whose last tile has inc,
//      or the left edge (+inf), composed with the gag maps in between.
// Every wait is on tiles with smaller tickets.
__device__ uint32_t look_back(int32_t tile, int32_t ntiles, int32_t i, int32_t m, Map total,
                              uint64_t* __restrict__ flags, uint32_t* __restrict__ ctrl) {
  const int lane = threadIdx.x & 63;
  const int32_t ngroups = (ntiles + kLookback - 1) / kLookback;
  uint64_t* agg = flags + (int64_t)i * ntiles;
  const uint64_t* inc = flags + ((int64_t)m + i) * ntiles;
  uint64_t* gag = flags + 2 * (int64_t)m * ntiles + (int64_t)i * ngroups;
  if (lane == 0) store_flag(&agg[tile], pack_agg(total));
  if (tile == 0) return kInf;  // gamma(i, 0) = +inf

  const int32_t first = tile & ~(kLookback - 1);
  const bool closer = tile - first == kLookback - 1;  // last tile of its group
  uint32_t spins = 0;
  Map acc{kInf, 0};  // maps of this group's tiles left of `tile`
  if (tile > first) {
    while (true) {
      const int32_t p = tile - 1 - lane;
      const bool valid = p >= first;
      const uint64_t wa = valid ? load_flag(&agg[p]) : 0ull;
      const uint64_t wi = valid ? load_flag(&inc[p]) : 0ull;
      const uint64_t inclm = __ballot(valid && (wi & 3u) == kIncl);
      const uint64_t readym = __ballot(valid && (wa & 3u) == kAgg);
      const uint64_t validm = __ballot(valid);
      const int kn = inclm ? __builtin_ctzll(inclm) : 64;  // nearest with inc
      const int k = closer ? 64 : kn;                       // lanes to compose
      const uint64_t need = (k < 64 ? (1ull << k) - 1 : ~0ull) & validm;
      if ((readym & need) != need) {
        if (give_up(spins, ctrl)) return kInf;
        continue;
      }
      const Map win = wave_compose(lane < k && valid ? unpack_agg(wa) : Map{kInf, 0});
      if (closer && lane == 0) store_flag(&gag[tile / kLookback], pack_agg(compose_sat(win, total)));
      if (kn < 64) {
        const Map part = closer ? wave_compose(lane < kn ? unpack_agg(wa) : Map{kInf, 0}) : win;
        const uint32_t v = (uint32_t)__shfl((int)(uint32_t)(wi >> 32), kn);
        return min(part.a, v + part.d);
      }
      acc = win;
      break;
    }
  }
  // 2. groups to the left of this tile's group
  int32_t gbase = first / kLookback - 1;
  Map gacc{kInf, 0};
  while (true) {
    const int32_t g = gbase - lane;
    const bool valid = g >= 0;
    const uint64_t wa = valid ? load_flag(&gag[g]) : 0ull;
    const uint64_t wi = valid ? load_flag(&inc[(int64_t)g * kLookback + kLookback - 1]) : 0ull;
    const uint64_t inclm = __ballot(valid && (wi & 3u) == kIncl);
    const uint64_t readym = __ballot(valid && (wa & 3u) == kAgg);
    int k = inclm ? __builtin_ctzll(inclm) : 64;
    const bool edge = gbase + 1 < 64 && gbase + 1 < k;  // the left edge comes first
    if (edge) k = gbase + 1;
    const uint64_t need = k < 64 ? (1ull << k) - 1 : ~0ull;
    if ((readym & need) != need) {
      if (give_up(spins, ctrl)) return kInf;
      continue;
    }
    gacc = compose_sat(wave_compose(lane < k ? unpack_agg(wa) : Map{kInf, 0}), gacc);
    if (k < 64) {
      const uint32_t v = edge ? kInf : (uint32_t)__shfl((int)(uint32_t)(wi >> 32), k);
      const uint32_t xg = min(gacc.a, v + gacc.d);
      return min(acc.a, xg + acc.d);
    }
    gbase -= 64;
  }
}

// ROW: a resident row to extend (row_in) or to write (compiled apart, so
// that the single-query form keeps its registers and so its tiles per CU).
template <int C, bool LowReg, bool ROW>
__global__ __launch_bounds__(kWideThreads, LowReg ? 3 : 1) void k_align_wide(
    const uint32_t* __restrict__ ref, int64_t n, int32_t ntiles, const int16_t* __restrict__ q,
    int32_t m, uint64_t* __restrict__ flags, uint64_t* __restrict__ tile_key,
    uint32_t* __restrict__ ctrl, uint32_t* __restrict__ row, int row_in,
    const uint64_t* __restrict__ left_of_tile) {
  constexpr int T = kWideThreads * C;
  __shared__ uint32_t sa[kWideThreads / 64], sd[kWideThreads / 64];
  __shared__ uint32_t lastcol[2][kWideThreads];
  __shared__ uint32_t s_x;
  __shared__ int32_t s_tile;
  __shared__ uint64_t sk[kWideThreads / 64];

  if (threadIdx.x == 0) s_tile = (int32_t)atomicAdd(&ctrl[0], 1u);
  __syncthreads();
  const int32_t tile = s_tile;
  const int64_t col0 = (int64_t)tile * T + (int64_t)threadIdx.x * C;

  uint32_t y[C], prev[C];
#pragma unroll
  for (int c = 0; c < C; ++c) {
    y[c] = col0 + c < n ? ref[col0 + c] : 0u;
    prev[c] = 0u;  // gamma(0, j) = 0
  }
  // gamma(i-1, first column of the tile - 1); row 0: 0, or the resident
  // row's value left of the tile (+inf left of column 0)
  uint32_t xprev = 0u;
  // the first row's diagonal of this thread's first cell
  uint32_t left_first = 0u;
  if constexpr (ROW) {
    if (row_in) {
      if (col0 + C <= n) {  // the whole strip: 16-byte loads (col0 is a multiple of 8)
#pragma unroll
        for (int c = 0; c < C; c += 4) {
          const uint4 v = *(const uint4*)(row + col0 + c);
          prev[c] = v.x;
          prev[c + 1] = v.y;
          prev[c + 2] = v.z;
          prev[c + 3] = v.w;
        }
      } else {
#pragma unroll
        for (int c = 0; c < C; ++c)
          if (col0 + c < n) prev[c] = row[col0 + c];
      }
      xprev = tile == 0 ? kInf : (uint32_t)left_of_tile[tile];
      if (threadIdx.x > 0 && col0 - 1 < n) left_first = row[col0 - 1];  // in this tile
    }
  }

  for (int32_t i = 0; i < m; ++i) {
    const uint32_t x = (uint32_t)((int32_t)q[i] + (int32_t)kI16Bias);
    const uint32_t left0 =
        threadIdx.x == 0 ? xprev : (i == 0 ? left_first : lastcol[(i - 1) & 1][threadIdx.x - 1]);

    // 1. this thread's map
    Map mine{kInf, 0};
    {
      uint32_t left = left0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const uint32_t a = cell_a<LowReg>(x, y[c], left, prev[c]);
        mine.a = min(a, sad<LowReg>(x, y[c], mine.a));
        mine.d = sad<LowReg>(x, y[c], mine.d);
        left = prev[c];
      }
    }
    // 2. maps left of this thread, and the tile's
    Map total;
    const Map before = scan_maps(mine, total, sa, sd);

    // 3. publish, look back, publish (wave 0; see look_back)
    if (threadIdx.x < 64) {
      const uint32_t xin = look_back(tile, ntiles, i, m, total, flags, ctrl);
      if (threadIdx.x == 0) {
        const uint32_t last = min(total.a, xin + total.d);
        store_flag(&flags[((int64_t)m + i) * ntiles + tile], ((uint64_t)last << 32) | kIncl);
        s_x = xin;
      }
    }
    __syncthreads();
    const uint32_t xin = s_x;

    // 4. the row
    {
      uint32_t carry = min(before.a, xin + before.d);
      uint32_t left = left0;
#pragma unroll
      for (int c = 0; c < C; ++c) {
        const uint32_t a = cell_a<LowReg>(x, y[c], left, prev[c]);
        left = prev[c];
        carry = min(a, sad<LowReg>(x, y[c], carry));
        prev[c] = carry;
      }
    }
    lastcol[i & 1][threadIdx.x] = prev[C - 1];
    xprev = xin;
    __syncthreads();
  }

  // the new resident row (every thread of the tile has read its old values:
  // the loop's barriers lie between)
  if constexpr (ROW) {
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (col0 + c < n) row[col0 + c] = prev[c];
  }

  // last row: the first column with the minimum in this tile
  uint64_t k = ~0ull;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    const uint64_t kk = ((uint64_t)prev[c] << 32) | (uint64_t)(uint32_t)(col0 + c);
    if (col0 + c < n && kk < k) k = kk;
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)k, off);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(k >> 32), off);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    k = o < k ? o : k;
  }
  if ((threadIdx.x & 63) == 0) sk[threadIdx.x >> 6] = k;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kWideThreads / 64; ++w) k = sk[w] < k ? sk[w] : k;
    tile_key[tile] = k;
  }
}

// Flags and the ticket cleared for the next launch (a kernel, not a memset,
// so that the call can be captured in a graph); when a resident row is
// extended, the old value left of every tile (T columns each) copied aside.
__global__ void k_wide_clear(uint64_t* __restrict__ flags, int64_t nflags,
                             uint32_t* __restrict__ ctrl, const uint32_t* __restrict__ row,
                             int64_t T, int32_t ntiles, uint64_t* __restrict__ left_of_tile) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nflags) flags[i] = 0;
  if (i < 2) ctrl[i] = 0;
  if (row && i < ntiles) left_of_tile[i] = i > 0 ? row[i * T - 1] : 0u;
}

__global__ __launch_bounds__(kWideThreads) void k_wide_final(const uint64_t* __restrict__ tile_key,
                                                             int32_t ntiles,
                                                             const uint32_t* __restrict__ ctrl,
                                                             int32_t* cost, int32_t* end) {
  __shared__ uint64_t sk[kWideThreads / 64];
  uint64_t k = ~0ull;
  for (int32_t t = threadIdx.x; t < ntiles; t += kWideThreads) k = tile_key[t] < k ? tile_key[t] : k;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)k, off);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(k >> 32), off);
    const uint64_t o = ((uint64_t)hi << 32) | lo;
    k = o < k ? o : k;
  }
  if ((threadIdx.x & 63) == 0) sk[threadIdx.x >> 6] = k;
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kWideThreads / 64; ++w) k = sk[w] < k ? sk[w] : k;
    const bool aborted = ctrl[1] != 0;
    *cost = aborted ? -1 : (int32_t)(uint32_t)(k >> 32);
    *end = aborted ? -1 : (int32_t)(uint32_t)k;
  }
}

// Tiles of one launch that are resident at once on the current device.
int resident_tiles(const void* fn) {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWideThreads, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

template <int C, bool LowReg, bool ROW>
hipError_t launch_c(const uint32_t* ref, int64_t n, const int16_t* q, int32_t m,
                    uint64_t* scratch, int32_t* cost, int32_t* end, hipStream_t st,
                    uint32_t* row, bool row_in) {
  const int64_t T = (int64_t)kWideThreads * C;
  const int32_t ntiles = (int32_t)((n + T - 1) / T);
  const int64_t ngroups = (ntiles + kLookback - 1) / kLookback;
  const int64_t nflags = 2 * (int64_t)m * ntiles + (int64_t)m * ngroups;
  uint64_t* flags = scratch;
  uint64_t* tile_key = flags + nflags;
  uint32_t* ctrl = (uint32_t*)(tile_key + ntiles);
  uint64_t* left_of_tile = tile_key + ntiles + 1;  // after the two control words
  // (nflags >= 2 * ntiles: the clearing grid covers every tile)
  hipLaunchKernelGGL(k_wide_clear, dim3((unsigned)((nflags + 255) / 256)), dim3(256), 0, st,
                     flags, nflags, ctrl, row_in ? row : nullptr, T, ntiles, left_of_tile);
  hipLaunchKernelGGL((k_align_wide<C, LowReg, ROW>), dim3((unsigned)ntiles), dim3(kWideThreads), 0,
                     st, ref, n, ntiles, q, m, flags, tile_key, ctrl, row, row_in ? 1 : 0,
                     left_of_tile);
  hipLaunchKernelGGL(k_wide_final, dim3(1), dim3(kWideThreads), 0, st, tile_key, ntiles, ctrl,
                     cost, end);
  return hipGetLastError();
}

}  // namespace

int wide_pick_cols(int64_t n, int device) {
  // Narrow tiles keep each thread's two sweeps of a row short, but every
  // tile adds flag traffic, and tiles beyond those resident at once run in
  // further rounds.  Measured on MI355X (250 rows): the narrowest width with
  // at most 64 tiles (one look-back window) is fastest up to a few hundred
  // thousand columns, then the narrowest with at most 256 tiles; beyond
  // that, 32 columns per thread (whose low-register form keeps the most
  // columns resident).
  (void)device;
  const int cols[4] = {8, 16, 32, 64};
  for (int64_t limit : {int64_t(kLookback), int64_t(256)})
    for (int k = 0; k < 4; ++k)
      if (wide_tiles(n, cols[k]) <= limit) return cols[k];
  return 32;
}

int64_t wide_noalloc_words() { return kNoallocWords; }

hipError_t wide_noalloc_scratch(int device, uint64_t** out) {
  constexpr int kDevices = 64;
  static std::mutex mu;
  static uint64_t* addr[kDevices] = {};
  if (device < 0 || device >= kDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(mu);
  if (!addr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(g_noalloc_scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    addr[device] = (uint64_t*)p;
  }
  *out = addr[device];
  return hipSuccess;
}

int64_t wide_tiles(int64_t n, int cols) { return (n + (int64_t)kWideThreads * cols - 1) /
                                                 ((int64_t)kWideThreads * cols); }

int64_t wide_scratch_words(int64_t n, int32_t m, int cols) {
  const int64_t t = wide_tiles(n, cols);
  const int64_t g = (t + kLookback - 1) / kLookback;
  // flags, tile keys, two control words, the resident row's values left of
  // every tile
  return 2 * (int64_t)m * t + (int64_t)m * g + t + 1 + t;
}

namespace {

template <bool ROW>
hipError_t launch_row(const uint32_t* ref, int64_t n, const int16_t* q, int32_t m, int cols,
                      uint64_t* scratch, int32_t* cost, int32_t* end, hipStream_t st,
                      uint32_t* row, bool row_in) {
  switch (cols) {
    case 8: return launch_c<8, false, ROW>(ref, n, q, m, scratch, cost, end, st, row, row_in);
    case 16: return launch_c<16, false, ROW>(ref, n, q, m, scratch, cost, end, st, row, row_in);
    case 32: {
      // the low-register form when the plain one would run in more rounds
      if (wide_tiles(n, 32) > resident_tiles((const void*)k_align_wide<32, false, ROW>))
        return launch_c<32, true, ROW>(ref, n, q, m, scratch, cost, end, st, row, row_in);
      return launch_c<32, false, ROW>(ref, n, q, m, scratch, cost, end, st, row, row_in);
    }
    case 64: return launch_c<64, false, ROW>(ref, n, q, m, scratch, cost, end, st, row, row_in);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_align_wide(const uint32_t* ref, int64_t n, const int16_t* q, int32_t m,
                             int cols, uint64_t* scratch, int32_t* cost, int32_t* end,
                             hipStream_t st, uint32_t* row, bool row_in) {
  if (n < 1 || m < 1 || wide_tiles(n, cols) > INT_MAX || (row_in && !row))
    return hipErrorInvalidValue;
  return row ? launch_row<true>(ref, n, q, m, cols, scratch, cost, end, st, row, row_in)
             : launch_row<false>(ref, n, q, m, cols, scratch, cost, end, st, row, row_in);
}

}  // namespace sdtw
