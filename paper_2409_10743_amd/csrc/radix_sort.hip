// Stable LSD radix sort of (u64 key, u32 value) pairs for the Morton codes
// of section 4.2.2 (64-bit codes make the sort "slightly" slower than 32-bit
// ones; here it is 8 passes of 8-bit digits over 63 used bits).
//
// The clustering call's sort moves 32-bit key words instead: the passes
// over the low half of the codes carry the high half as a second 32-bit
// word beside the value, the last of them keeps only the high half, and
// the passes over the high half move it alone (8 instead of 12 bytes per
// element and pass, and 36 instead of 53 KB of LDS per block: four blocks
// per CU instead of three).  The sorted codes themselves are not written:
// the build's first level recomputes each leaf's code from its point.
//
// One kernel per digit pass ("onesweep"): every workgroup takes the next
// tile id from an atomic counter, ranks its 4096 keys by digit in LDS,
// publishes its per-digit counts, and finds the counts of all earlier tiles
// by decoupled look-back.  Tile ids come from the counter, not blockIdx, so
// a tile only ever waits on tiles that are already running: the wait always
// ends.  It is also bounded: a stalled wait flags the run as failed rather
// than spinning forever.  Keys and values are staged in LDS in digit order
// so the global writes go out as runs of consecutive addresses.
#include <algorithm>
#include <cstdlib>
#include <type_traits>

#include "pipeline.hpp"

namespace dbx {

namespace {

constexpr int WAVES = SORT_THREADS / 64;
constexpr uint32_t ST_AGG = 1u << 30;   // tile's own count published
constexpr uint32_t ST_INC = 2u << 30;   // inclusive prefix published
constexpr uint32_t ST_VAL = (1u << 30) - 1;
constexpr uint32_t SPIN_LIMIT = 1u << 22;
constexpr int LOOKBACK = 4;  // predecessor tiles read per look-back round trip

// Exclusive prefix sum of one value per thread over a 256-thread block.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* s_tmp) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) s_tmp[wave] = x;
  __syncthreads();
  uint32_t add = 0;
  for (int w = 0; w < wave; ++w) add += s_tmp[w];
  __syncthreads();
  return x - v + add;
}

__global__ __launch_bounds__(256) void k_digit_hist(const uint64_t* __restrict__ keys,
                                                   uint32_t n, uint32_t* __restrict__ hist) {
  __shared__ uint32_t sh[SORT_PASSES * RADIX];
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x) sh[t] = 0;
  __syncthreads();
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint64_t k = keys[i];
#pragma unroll
    for (int p = 0; p < SORT_PASSES; ++p)
      atomicAdd(&sh[p * RADIX + ((k >> (8 * p)) & 0xff)], 1u);
  }
  __syncthreads();
  for (int t = threadIdx.x; t < SORT_PASSES * RADIX; t += blockDim.x)
    if (sh[t]) atomicAdd(&hist[t], sh[t]);
}

// With `drop` (not null) the pass reads the number of low code bits the
// keys cleared: a pass below it returns at once, and the passes that run
// alternate between the two buffer pairs so that the last ends in (ka, va):
// the codes start in ka if an even number of passes is skipped, else in kb.
//
// KIN is the key word the pass reads (the whole u64 code, or a 32-bit half
// of it); `shift` is the digit's position in that word and `pass` the
// digit's number in the 64-bit code.  PAY: a second 32-bit word travels
// with each key (u32 words n..2n-1 of the key buffers: the high half while
// the low half is sorted).  NARROW: the pass writes that word as the
// output key and no second word (the last pass over the low half).
//
// skip_lo (8: never): a pass from skip_lo on whose digit is the same for
// every key is skipped, not copied, when it pairs with a neighbouring such
// pass: in each run of consecutive one-digit passes the first and second
// are skipped, the third and fourth, and so on (an odd run's last pass
// still copies).  A skipped pair leaves the data where the host's
// alternation expects it after both, so no direction changes.  ghist is
// this pass's row of the digit counts of all passes.
template <bool IOTA, int ITEMS, class KIN, bool PAY, bool NARROW>
__global__ __launch_bounds__(SORT_THREADS) void k_onesweep(
    uint64_t* ka, uint64_t* kb, uint32_t* va, uint32_t* vb, uint32_t n, int shift, int pass_no,
    int skip_lo, const uint32_t* __restrict__ drop, const uint32_t* __restrict__ ghist,
    uint32_t* __restrict__ status, uint32_t* __restrict__ next_status,
    uint32_t* __restrict__ tile_ctr, uint32_t* __restrict__ err) {
  static_assert(!NARROW || PAY, "a narrowing pass writes the carried word");
  using KOUT = typename std::conditional<NARROW, uint32_t, KIN>::type;
  constexpr int TILE = SORT_THREADS * ITEMS;
  __shared__ KIN s_keys[TILE];                // keys and values in digit order
  __shared__ uint32_t s_vals[TILE];
  __shared__ uint32_t s_pay[PAY ? TILE : 1];  // the carried words, likewise
  // per-wave digit counts, then each wave's first slot per digit in the
  // tile; after staging, row 0 holds the global offset minus the tile offset
  __shared__ uint32_t s_whist[WAVES][RADIX];
  __shared__ uint32_t s_tmp[WAVES];
  __shared__ uint32_t s_tile;
  __shared__ uint32_t s_one;  // bit q: every key has the same digit in pass q

  // the next pass's look-back words start at zero: each workgroup clears
  // one tile's row of them (the grid has one workgroup per tile), also in a
  // pass that returns at once below
  if (next_status) next_status[size_t(blockIdx.x) * RADIX + threadIdx.x] = 0u;
  uint64_t* bin = ka;  // without `drop`: (ka, va) -> (kb, vb)
  uint64_t* bout = kb;
  const uint32_t* vin = va;
  uint32_t* vout = vb;
  bool iota = IOTA;
  if (drop) {
    const int skip = int(*drop) / 8;
    if (pass_no < skip) return;
    const bool from_a = ((pass_no - skip) % 2 == 0) == (skip % 2 == 0);
    if (!from_a) {
      bin = kb;
      bout = ka;
      vin = vb;
      vout = va;
    }
    iota = pass_no == skip;
  }
  const KIN* kin = reinterpret_cast<const KIN*>(bin);
  KOUT* kout = reinterpret_cast<KOUT*>(bout);
  const uint32_t* pin = reinterpret_cast<const uint32_t*>(bin) + n;
  uint32_t* pout = reinterpret_cast<uint32_t*>(bout) + n;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t gcount = ghist[tid];  // this pass's count of digit tid
  if (skip_lo < SORT_PASSES) {
    if (tid == 0) s_one = 0;
    __syncthreads();
    const uint32_t* all = ghist - size_t(pass_no) * RADIX;  // every pass's counts
    uint32_t mine = 0;
    for (int q = skip_lo; q < SORT_PASSES; ++q)
      mine |= all[size_t(q) * RADIX + tid] == n ? (1u << q) : 0u;
    if (mine) atomicOr(&s_one, mine);
    __syncthreads();
    const uint32_t one = s_one;
    if (pass_no >= skip_lo && ((one >> pass_no) & 1u)) {
      int a = pass_no;  // the run of one-digit passes holding this one
      while (a - 1 >= skip_lo && ((one >> (a - 1)) & 1u)) --a;
      const bool second = ((pass_no - a) & 1) != 0;
      const bool paired = second || (pass_no + 1 < SORT_PASSES && ((one >> (pass_no + 1)) & 1u));
      if (paired) return;  // (uniform: every thread reads the same bits)
    }
  }
  if (tid == 0) s_tile = atomicAdd(tile_ctr, 1u);
  for (int w = 0; w < WAVES; ++w) s_whist[w][tid] = 0;
  // one digit for every key (constant code bits, or a set id shared by all
  // keys): the pass keeps the order, so each tile only copies itself
  const bool trivial = __syncthreads_or(gcount == n);
  const uint32_t tile = s_tile;
  const uint32_t tile_base = tile * TILE;
  const uint32_t wbase = tile_base + wave * (64 * ITEMS);

  KIN key[ITEMS];
  uint32_t val[ITEMS];  // loaded with the keys, early: its latency hides behind the ranking
  uint32_t pay[ITEMS];
  uint32_t rank[ITEMS];
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));

#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    uint32_t idx = wbase + k * 64 + lane;
    key[k] = idx < n ? kin[idx] : KIN(~KIN(0));
    val[k] = iota ? idx : (idx < n ? vin[idx] : 0u);
    pay[k] = PAY && idx < n ? pin[idx] : 0u;
  }
  if (trivial) {  // all loads above are in flight: write them back where they were
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
      const uint32_t idx = wbase + k * 64 + lane;
      if (idx < n) {
        kout[idx] = NARROW ? KOUT(pay[k]) : KOUT(key[k]);
        vout[idx] = val[k];
        if (PAY && !NARROW) pout[idx] = pay[k];
      }
    }
    return;
  }

  // rank each key among the keys of this wave with the same digit; the
  // order of keys inside a wave is (item, lane), i.e. their input order
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    uint32_t idx = wbase + k * 64 + lane;
    bool ok = idx < n;
    uint32_t d = uint32_t(key[k] >> shift) & 0xff;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      uint64_t m = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? m : ~m;
    }
    int leader = ok ? 63 - __clzll(peers) : lane;
    uint32_t old = 0;
    if (ok && lane == leader) {
      old = s_whist[wave][d];
      s_whist[wave][d] = old + __popcll(peers);
    }
    old = __shfl(old, leader, 64);
    rank[k] = old + __popcll(peers & lt_mask);
  }
  __syncthreads();

  // per digit (one thread each): wave prefixes, tile count, look-back
  const int d = tid;
  uint32_t total = 0;
#pragma unroll
  for (int w = 0; w < WAVES; ++w) {
    uint32_t c = s_whist[w][d];
    s_whist[w][d] = total;
    total += c;
  }
  uint32_t excl = 0;
  uint32_t* st = status + size_t(tile) * RADIX + d;
  if (tile == 0) {
    st_agent(st, ST_INC | total);
  } else {
    st_agent(st, ST_AGG | total);
    // look back LOOKBACK tiles per round trip: their words are read
    // together, then taken in order up to the first inclusive prefix (done)
    // or the first tile that has published nothing yet (read again from
    // there after a pause)
    int32_t j = int32_t(tile) - 1;
    uint32_t spins = 0;
    for (;;) {
      uint32_t v[LOOKBACK];
#pragma unroll
      for (int q = 0; q < LOOKBACK; ++q)
        v[q] = j - q >= 0 ? ld_agent(status + size_t(j - q) * RADIX + d) : ST_INC;
      int taken = 0;
      bool done = false;
#pragma unroll
      for (int q = 0; q < LOOKBACK; ++q) {
        const uint32_t f = v[q] & ~ST_VAL;
        if (done || f == 0 || taken < q) continue;  // stop at the first unpublished tile
        excl += v[q] & ST_VAL;
        done = f == ST_INC;
        taken = q + 1;
      }
      if (done) break;
      j -= taken;
      if (taken < LOOKBACK) {
        if (++spins > SPIN_LIMIT) { atomicOr(err, STATUS_SORT_STALL); break; }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    st_agent(st, ST_INC | ((excl + total) & ST_VAL));
  }
  // global digit start for this pass: exclusive scan of the digit counts
  uint32_t gstart = block_exclusive_scan(gcount, s_tmp);
  uint32_t loff = block_exclusive_scan(total, s_tmp);
  for (int w = 0; w < WAVES; ++w) s_whist[w][d] += loff;
  __syncthreads();

  // stage keys and values in digit order, then write runs of equal digits
#pragma unroll
  for (int k = 0; k < ITEMS; ++k) {
    const uint32_t idx = wbase + k * 64 + lane;
    if (idx < n) {
      const uint32_t dd = uint32_t(key[k] >> shift) & 0xff;
      const uint32_t p = s_whist[wave][dd] + rank[k];
      s_keys[p] = key[k];
      s_vals[p] = val[k];
      if (PAY) s_pay[p] = pay[k];
    }
  }
  __syncthreads();
  // the per-wave slots are no longer needed: row 0 now holds the offsets
  // (keeps LDS at 53 KB for 64-bit keys, three blocks per CU)
  s_whist[0][d] = gstart + excl - loff;
  __syncthreads();
  const uint32_t* s_base = s_whist[0];
  const uint32_t tile_n = min(uint32_t(TILE), n - tile_base);
  for (uint32_t p = tid; p < tile_n; p += SORT_THREADS) {
    const KIN kk = s_keys[p];
    const uint32_t dst = s_base[uint32_t(kk >> shift) & 0xff] + p;
    if (dst < n) {  // always true unless a look-back wait was cut short
      kout[dst] = NARROW ? KOUT(s_pay[p]) : KOUT(kk);
      vout[dst] = s_vals[p];
      if (PAY && !NARROW) pout[dst] = s_pay[p];
    }
  }
}

}  // namespace

void launch_digit_histogram(const uint64_t* keys, uint32_t n, uint32_t* hist,
                            hipStream_t s) {
  if (n == 0) return;
  uint32_t blocks = std::min((n + 255) / 256, 2048u);
  hipLaunchKernelGGL(k_digit_hist, dim3(blocks), dim3(256), 0, s, keys, n, hist);
}


namespace {
// The word layouts a pass can move (see k_onesweep): whole 64-bit codes;
// the low half with the high half carried (LO), the last such pass (LO_LAST,
// which keeps only the high half); the high half alone (HI).
enum PassWords { WIDE = 0, LO = 1, LO_LAST = 2, HI = 3 };

template <bool IOTA, int ITEMS>
void launch_pass(int words, dim3 grid, uint64_t* ka, uint64_t* kb, uint32_t* va, uint32_t* vb,
                 uint32_t n, int p, int skip_lo, const uint32_t* drop, const uint32_t* ghist,
                 uint32_t* st, uint32_t* next, uint32_t* ctr, uint32_t* err, hipStream_t s) {
  const dim3 block(SORT_THREADS);
  if (words == LO)
    hipLaunchKernelGGL((k_onesweep<IOTA, ITEMS, uint32_t, true, false>), grid, block, 0, s, ka,
                       kb, va, vb, n, 8 * p, p, skip_lo, drop, ghist, st, next, ctr, err);
  else if (words == LO_LAST)
    hipLaunchKernelGGL((k_onesweep<IOTA, ITEMS, uint32_t, true, true>), grid, block, 0, s, ka,
                       kb, va, vb, n, 8 * p, p, skip_lo, drop, ghist, st, next, ctr, err);
  else if (words == HI)
    hipLaunchKernelGGL((k_onesweep<IOTA, ITEMS, uint32_t, false, false>), grid, block, 0, s, ka,
                       kb, va, vb, n, 8 * p - 32, p, skip_lo, drop, ghist, st, next, ctr, err);
  else
    hipLaunchKernelGGL((k_onesweep<IOTA, ITEMS, uint64_t, false, false>), grid, block, 0, s, ka,
                       kb, va, vb, n, 8 * p, p, skip_lo, drop, ghist, st, next, ctr, err);
}

// one pass from (kin, vin) to (kout, vout); with `drop`, the kernel picks
// the direction itself (see k_onesweep)
// st: this pass's look-back words (zero); the next pass's, if any, follow
// them and are cleared here
template <int ITEMS>
void sort_pass(bool iota, int words, const uint64_t* kin, uint64_t* kout, const uint32_t* vin,
               uint32_t* vout, uint32_t n, int p, int skip_lo, const uint32_t* drop,
               const SortScratch& sc, uint32_t* st, hipStream_t s) {
  uint32_t* next = p + 1 < SORT_PASSES ? st + size_t(sort_tiles(n, ITEMS)) * RADIX : nullptr;
  const uint32_t tiles = sort_tiles(n, ITEMS);
  uint64_t* ka = const_cast<uint64_t*>(kin);  // read-only in this direction
  uint32_t* va = const_cast<uint32_t*>(vin);
  if (iota)
    launch_pass<true, ITEMS>(words, dim3(tiles), ka, kout, va, vout, n, p, skip_lo, drop,
                             sc.hist + p * RADIX, st, next, sc.tile_ctr + p, sc.err, s);
  else
    launch_pass<false, ITEMS>(words, dim3(tiles), ka, kout, va, vout, n, p, skip_lo, drop,
                              sc.hist + p * RADIX, st, next, sc.tile_ctr + p, sc.err, s);
}

}  // namespace

bool launch_radix_sort(uint64_t* ka, uint64_t* kb, uint32_t* va, uint32_t* vb,
                       uint32_t n, int first_pass, bool iota_vals,
                       const SortScratch& sc, hipStream_t s,
                       void (*after_pass)(void*, int), void* arg, int tile_items) {
  bool in_a = true;
  if (n == 0) return true;
  const int items = tile_items ? tile_items : SORT_ITEMS;
  const uint32_t words = sort_tiles(n, items) * RADIX;
  for (int p = first_pass; p < SORT_PASSES; ++p) {
    const uint64_t* kin = in_a ? ka : kb;
    uint64_t* kout = in_a ? kb : ka;
    const uint32_t* vin = in_a ? va : vb;
    uint32_t* vout = in_a ? vb : va;
    uint32_t* st = sc.status + size_t(p - first_pass) * words;  // the first pass's: zeroed
    const bool iota = p == first_pass && iota_vals;
    // one-digit passes are skipped in pairs, never the one that makes the values
    const int lo = first_pass + (iota_vals ? 1 : 0);
    if (items == 8) sort_pass<8>(iota, WIDE, kin, kout, vin, vout, n, p, lo, nullptr, sc, st, s);
    else if (items == 12) sort_pass<12>(iota, WIDE, kin, kout, vin, vout, n, p, lo, nullptr, sc, st, s);
    else sort_pass<16>(iota, WIDE, kin, kout, vin, vout, n, p, lo, nullptr, sc, st, s);
    if (after_pass) after_pass(arg, p);
    in_a = !in_a;
  }
  return in_a;
}

void launch_radix_sort_dropped(uint64_t* ka, uint64_t* kb, uint32_t* va, uint32_t* vb,
                               uint32_t n, const uint32_t* drop, const SortScratch& sc,
                               hipStream_t s, void (*after_pass)(void*, int), void* arg,
                               int tile_items) {
  if (n == 0) return;
  const int items = tile_items ? tile_items : SORT_ITEMS;
  const uint32_t words = sort_tiles(n, items) * RADIX;
  for (int p = 0; p < SORT_PASSES; ++p) {
    uint32_t* st = sc.status + size_t(p) * words;
    const int w = p < 3 ? LO : p == 3 ? LO_LAST : HI;
    if (items == 8) sort_pass<8>(false, w, ka, kb, va, vb, n, p, SORT_PASSES, drop, sc, st, s);
    else if (items == 12) sort_pass<12>(false, w, ka, kb, va, vb, n, p, SORT_PASSES, drop, sc, st, s);
    else sort_pass<16>(false, w, ka, kb, va, vb, n, p, SORT_PASSES, drop, sc, st, s);
    if (after_pass) after_pass(arg, p);
  }
}

}  // namespace dbx
