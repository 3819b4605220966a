// primitives.h -- the device-wide primitives of the paper's evaluation loop
// (the ablation of Sections 3.4-3.5): inclusive prefix sum, stream compaction
// of an array (the removal of dummy equations), stable LSD radix sort of
// (32-bit key, 64-bit value) pairs (the sort of the equations by variable), and
// reduce by key over runs of equal adjacent keys (the merge of
// communication-eligible equations).  Each primitive is a few kernels over
// tiles of 2048 elements (256 threads x 8 items) with a prefix sum over the
// per-tile counts between them; temporary device memory comes from the
// caller's Scratch.  A single tile takes one launch per primitive (the
// sort runs all its passes in LDS).
#ifndef INET_PRIMITIVES_H
#define INET_PRIMITIVES_H

#include <hip/hip_runtime.h>

#include <cstdint>

namespace inet {
namespace prim {

constexpr int BLOCK = 256;
constexpr int ITEMS = 8;
constexpr int TILE = BLOCK * ITEMS;
constexpr int WAVES = BLOCK / 64;

inline int tiles_of(size_t n) { return (int)((n + TILE - 1) / TILE); }

// temporary device memory of the primitives: a bump arena over one device
// buffer, emptied by the caller between calls
struct Scratch {
  char *base = nullptr;
  size_t size = 0, used = 0;
  int take(size_t bytes, void **out) {
    const size_t b = (bytes + 255) & ~size_t(255);
    if (!base || used + b > size) return -1;
    *out = base + used;
    used += b;
    return 0;
  }
  void reset() { used = 0; }
};

// arena bytes that one call on n elements may take (the radix sort's
// histograms and every level of the prefix sums over per-tile counts)
inline size_t scratch_bytes(size_t n) {
  const size_t t = (n + TILE - 1) / TILE + 1;
  return 2 * (4 * (size_t)256 * t) + 16 * t + ((size_t)1 << 20);
}

// --- wave and block sums -------------------------------------------------

template <class T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = __lane_id();
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const T o = __shfl_up(v, d, 64);
    if (lane >= d) v += o;
  }
  return v;
}

// exclusive prefix of v over the block, and the block total
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T *s_wave, T *total) {
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  const T incl = wave_incl_scan(v);
  if (lane == 63) s_wave[w] = incl;
  __syncthreads();
  T before = 0, all = 0;
#pragma unroll
  for (int k = 0; k < WAVES; k++) {
    const T x = s_wave[k];
    before += k < w ? x : T(0);
    all += x;
  }
  __syncthreads();
  *total = all;
  return before + incl - v;
}

// --- inclusive prefix sum ------------------------------------------------

// per-tile sums
template <class T>
__global__ __launch_bounds__(BLOCK) void k_tile_sum(const T *__restrict__ in, size_t n,
                                                    T *__restrict__ part) {
  __shared__ T s_wave[WAVES];
  const size_t base = (size_t)blockIdx.x * TILE;
  T s = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; k++) {
    const size_t i = base + (size_t)k * BLOCK + threadIdx.x;
    if (i < n) s += in[i];
  }
  T tot;
  (void)block_excl_scan(s, s_wave, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// inclusive scan of each tile, plus the exclusive prefix of the tiles before
// it (part_incl: inclusive prefix over tiles, or null for a single tile)
template <class T>
__global__ __launch_bounds__(BLOCK) void k_tile_scan(const T *__restrict__ in, T *__restrict__ out,
                                                     size_t n, const T *__restrict__ part_incl,
                                                     const T *__restrict__ part) {
  __shared__ T s_wave[WAVES];
  const size_t base = (size_t)blockIdx.x * TILE + (size_t)threadIdx.x * ITEMS;
  T v[ITEMS];
  T run = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; k++) {
    const size_t i = base + k;
    run += i < n ? in[i] : T(0);
    v[k] = run;
  }
  T tot;
  T off = block_excl_scan(run, s_wave, &tot);
  if (part_incl) off += part_incl[blockIdx.x] - part[blockIdx.x];
#pragma unroll
  for (int k = 0; k < ITEMS; k++) {
    const size_t i = base + k;
    if (i < n) out[i] = v[k] + off;
  }
}

// out[i] = in[0] + ... + in[i]
template <class T>
int inclusive_sum(const T *in, T *out, size_t n, Scratch &S, hipStream_t s) {
  if (n == 0) return 0;
  const int t = tiles_of(n);
  if (t == 1) {
    hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(BLOCK), 0, s, in, out, n, (const T *)nullptr,
                       (const T *)nullptr);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  T *part = nullptr, *part_incl = nullptr;
  if (S.take(sizeof(T) * t, (void **)&part) || S.take(sizeof(T) * t, (void **)&part_incl)) return -1;
  hipLaunchKernelGGL(k_tile_sum<T>, dim3(t), dim3(BLOCK), 0, s, in, n, part);
  if (inclusive_sum<T>(part, part_incl, (size_t)t, S, s)) return -1;
  hipLaunchKernelGGL(k_tile_scan<T>, dim3(t), dim3(BLOCK), 0, s, in, out, n,
                     (const T *)part_incl, (const T *)part);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// --- compaction: emit every index whose flag is set, in order --------------

template <class F>
__global__ __launch_bounds__(BLOCK) void k_flag_count(size_t n, F flag, uint32_t *__restrict__ cnt) {
  __shared__ uint32_t s_wave[WAVES];
  const size_t base = (size_t)blockIdx.x * TILE;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < ITEMS; k++) {
    const size_t i = base + (size_t)k * BLOCK + threadIdx.x;
    c += (i < n && flag(i)) ? 1u : 0u;
  }
  uint32_t tot;
  (void)block_excl_scan(c, s_wave, &tot);
  if (threadIdx.x == 0) cnt[blockIdx.x] = tot;
}

// emit(i, position) for each flagged i; positions follow the input order
// (cnt_incl / cnt: the tiles' inclusive and own counts, or null for a single
// tile, which then also writes the total)
template <class F, class E>
__global__ __launch_bounds__(BLOCK) void k_flag_emit(size_t n, F flag, E emit,
                                                     const uint32_t *__restrict__ cnt_incl,
                                                     const uint32_t *__restrict__ cnt,
                                                     int64_t *__restrict__ n_out) {
  __shared__ uint32_t s_wave[WAVES];
  const size_t base = (size_t)blockIdx.x * TILE;
  uint32_t off = cnt_incl ? cnt_incl[blockIdx.x] - cnt[blockIdx.x] : 0u;
  const int lane = __lane_id(), w = threadIdx.x >> 6;
  // rounds of BLOCK elements that hold any (the same in every thread)
  const size_t left = n - base;
  const int rounds = left >= (size_t)TILE ? ITEMS : (int)((left + BLOCK - 1) / BLOCK);
  for (int k = 0; k < rounds; k++) {
    const size_t i = base + (size_t)k * BLOCK + threadIdx.x;
    const bool f = i < n && flag(i);
    const unsigned long long m = __ballot(f ? 1 : 0);
    if (lane == 0) s_wave[w] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int q = 0; q < WAVES; q++) {
      before += q < w ? s_wave[q] : 0u;
      all += s_wave[q];
    }
    const uint32_t rank = (uint32_t)__builtin_amdgcn_mbcnt_hi(
        (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
    if (f) emit(i, (size_t)(off + before + rank));
    off += all;
    __syncthreads();
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0 && n_out)
    *n_out = (int64_t)(cnt_incl ? cnt_incl[blockIdx.x] : off);
}

// runs flag/emit over [0, n); the number emitted lands in *d_n_out (device)
template <class F, class E>
int compact(size_t n, F flag, E emit, int64_t *d_n_out, Scratch &S, hipStream_t s) {
  if (n == 0) {
    return hipMemsetAsync(d_n_out, 0, sizeof(int64_t), s) == hipSuccess ? 0 : -1;
  }
  const int t = tiles_of(n);
  if (t == 1) {  // one tile: one launch, which also counts
    hipLaunchKernelGGL((k_flag_emit<F, E>), dim3(1), dim3(BLOCK), 0, s, n, flag, emit,
                       (const uint32_t *)nullptr, (const uint32_t *)nullptr, d_n_out);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  uint32_t *cnt = nullptr, *incl = nullptr;
  if (S.take(4 * (size_t)t, (void **)&cnt) || S.take(4 * (size_t)t, (void **)&incl)) return -1;
  hipLaunchKernelGGL((k_flag_count<F>), dim3(t), dim3(BLOCK), 0, s, n, flag, cnt);
  if (inclusive_sum<uint32_t>(cnt, incl, (size_t)t, S, s)) return -1;
  hipLaunchKernelGGL((k_flag_emit<F, E>), dim3(t), dim3(BLOCK), 0, s, n, flag, emit,
                     (const uint32_t *)incl, (const uint32_t *)cnt, d_n_out);
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// keep the elements different from `drop`, in order
typedef unsigned long long u64w;
struct KeepIfNot {
  const u64w *in;
  u64w drop;
  __device__ bool operator()(size_t i) const { return in[i] != drop; }
};
struct CopyTo {
  const u64w *in;
  u64w *out;
  __device__ void operator()(size_t i, size_t p) const { out[p] = in[i]; }
};

inline int select_not(const u64w *in, u64w *out, size_t n, u64w drop, int64_t *d_n_out,
                      Scratch &S, hipStream_t s) {
  return compact(n, KeepIfNot{in, drop}, CopyTo{in, out}, d_n_out, S, s);
}

// --- stable LSD radix sort of (key, value) pairs, 8 bits per pass ----------

constexpr int RADIX = 256;

// per-tile histogram of one digit, stored digit-major: hist[d * tiles + tile]
__global__ __launch_bounds__(BLOCK) void k_rs_hist(const uint32_t *__restrict__ key, size_t n,
                                                   int shift, uint32_t *__restrict__ hist) {
  __shared__ uint32_t h[RADIX];
  h[threadIdx.x] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * TILE;
#pragma unroll
  for (int k = 0; k < ITEMS; k++) {
    const size_t i = base + (size_t)k * BLOCK + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = h[threadIdx.x];
}

// scatter each tile to the digit offsets; the order within a digit is the
// input order (ranks by wave match masks, waves and rounds in order)
template <class V>
__global__ __launch_bounds__(BLOCK) void k_rs_scatter(const uint32_t *__restrict__ key,
                                                      const V *__restrict__ val, size_t n,
                                                      int shift, const uint32_t *__restrict__ incl,
                                                      const uint32_t *__restrict__ hist,
                                                      uint32_t *__restrict__ key_out,
                                                      V *__restrict__ val_out) {
  __shared__ uint32_t run[RADIX];        // elements of each digit placed so far in this tile
  __shared__ uint32_t wcnt[WAVES][RADIX];  // this round's count of each digit per wave
  __shared__ uint32_t start[RADIX];      // first output position of each digit for this tile
  const int tid = threadIdx.x, w = tid >> 6;
  {
    const size_t j = (size_t)tid * gridDim.x + blockIdx.x;
    start[tid] = incl[j] - hist[j];
    run[tid] = 0;
    for (int q = 0; q < WAVES; q++) wcnt[q][tid] = 0;
  }
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * TILE;
  for (int k = 0; k < ITEMS; k++) {
    const size_t i = base + (size_t)k * BLOCK + tid;
    const bool valid = i < n;
    const uint32_t kk = valid ? key[i] : 0u;
    const uint32_t d = (kk >> shift) & 255u;
    // lanes of this wave holding the same digit
    unsigned long long same = __ballot(valid ? 1 : 0);
#pragma unroll
    for (int b = 0; b < 8; b++) {
      const unsigned long long m = __ballot(((d >> b) & 1u) ? 1 : 0);
      same &= ((d >> b) & 1u) ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__builtin_amdgcn_mbcnt_hi(
        (unsigned)(same >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)same, 0u));
    // the lowest lane of each digit group records the group's size
    if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (valid) {
      uint32_t before = 0;
      for (int q = 0; q < w; q++) before += wcnt[q][d];
      const uint32_t p = start[d] + run[d] + before + rank;
      key_out[p] = kk;
      val_out[p] = val[i];
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < WAVES; q++) {
      add += wcnt[q][tid];
      wcnt[q][tid] = 0;
    }
    run[tid] += add;
    __syncthreads();
  }
}

// one tile (n <= TILE) sorted by one block in LDS: the four passes of the
// sort above (digit counts, their exclusive prefix, the stable scatter in
// rounds of BLOCK elements) between two LDS buffers, one launch in all
template <class V>
__global__ __launch_bounds__(BLOCK) void k_rs_sort_tile(uint32_t *__restrict__ key,
                                                        V *__restrict__ val, int n) {
  __shared__ uint32_t sk[2][TILE];
  __shared__ V sv[2][TILE];
  __shared__ uint32_t run[RADIX], start[RADIX], s_wave[WAVES];
  __shared__ uint32_t wcnt[WAVES][RADIX];
  const int tid = threadIdx.x, w = tid >> 6;
  for (int i = tid; i < n; i += BLOCK) {
    sk[0][i] = key[i];
    sv[0][i] = val[i];
  }
  for (int pass = 0; pass < 4; pass++) {
    const int from = pass & 1, to = from ^ 1, shift = 8 * pass;
    run[tid] = 0;
    for (int q = 0; q < WAVES; q++) wcnt[q][tid] = 0;
    __syncthreads();
    for (int i = tid; i < n; i += BLOCK) atomicAdd(&run[(sk[from][i] >> shift) & 255u], 1u);
    __syncthreads();
    uint32_t tot;
    const uint32_t c = run[tid];
    start[tid] = block_excl_scan(c, s_wave, &tot);
    run[tid] = 0;
    __syncthreads();
    for (int k = 0; k * BLOCK < n; k++) {  // the rounds that hold any element
      const int i = k * BLOCK + tid;
      const bool valid = i < n;
      const uint32_t kk = valid ? sk[from][i] : 0u;
      const uint32_t d = (kk >> shift) & 255u;
      unsigned long long same = __ballot(valid ? 1 : 0);
#pragma unroll
      for (int b = 0; b < 8; b++) {
        const unsigned long long m = __ballot(((d >> b) & 1u) ? 1 : 0);
        same &= ((d >> b) & 1u) ? m : ~m;
      }
      const uint32_t rank = (uint32_t)__builtin_amdgcn_mbcnt_hi(
          (unsigned)(same >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)same, 0u));
      if (valid && rank == 0) wcnt[w][d] = (uint32_t)__popcll(same);
      __syncthreads();
      if (valid) {
        uint32_t before = 0;
        for (int q = 0; q < w; q++) before += wcnt[q][d];
        const uint32_t p = start[d] + run[d] + before + rank;
        sk[to][p] = kk;
        sv[to][p] = sv[from][i];
      }
      __syncthreads();
      uint32_t add = 0;
      for (int q = 0; q < WAVES; q++) {
        add += wcnt[q][tid];
        wcnt[q][tid] = 0;
      }
      run[tid] += add;
      __syncthreads();
    }
  }
  for (int i = tid; i < n; i += BLOCK) {  // four passes: the result is in buffer 0
    key[i] = sk[0][i];
    val[i] = sv[0][i];
  }
}

// sorts (key, val) by key, stably; the result is back in key / val (four
// passes through key_alt / val_alt, or in LDS for one tile)
template <class V>
int radix_sort_pairs(uint32_t *key, V *val, uint32_t *key_alt, V *val_alt, size_t n, Scratch &S,
                     hipStream_t s) {
  if (n <= 1) return 0;
  const int t = tiles_of(n);
  if (t == 1) {
    hipLaunchKernelGGL((k_rs_sort_tile<V>), dim3(1), dim3(BLOCK), 0, s, key, val, (int)n);
    return hipGetLastError() == hipSuccess ? 0 : -1;
  }
  uint32_t *hist = nullptr, *incl = nullptr;
  const size_t hn = (size_t)RADIX * t;
  if (S.take(4 * hn, (void **)&hist) || S.take(4 * hn, (void **)&incl)) return -1;
  uint32_t *ks[2] = {key, key_alt};
  V *vs[2] = {val, val_alt};
  for (int pass = 0; pass < 4; pass++) {
    const int from = pass & 1, to = from ^ 1;
    hipLaunchKernelGGL(k_rs_hist, dim3(t), dim3(BLOCK), 0, s, (const uint32_t *)ks[from], n,
                       8 * pass, hist);
    if (inclusive_sum<uint32_t>(hist, incl, hn, S, s)) return -1;
    hipLaunchKernelGGL((k_rs_scatter<V>), dim3(t), dim3(BLOCK), 0, s, (const uint32_t *)ks[from],
                       (const V *)vs[from], n, 8 * pass, (const uint32_t *)incl,
                       (const uint32_t *)hist, ks[to], vs[to]);
  }
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// --- reduce by key: each run of equal adjacent keys becomes one element, its
// values folded left to right with op ---------------------------------------

struct RunHead {
  const uint32_t *key;
  __device__ bool operator()(size_t i) const { return i == 0 || key[i] != key[i - 1]; }
};

template <class V, class Op>
struct FoldRun {
  const uint32_t *key;
  const V *val;
  size_t n;
  uint32_t *key_out;
  V *val_out;
  Op op;
  __device__ void operator()(size_t i, size_t p) const {
    const uint32_t k = key[i];
    V acc = val[i];
    for (size_t j = i + 1; j < n && key[j] == k; j++) acc = op(acc, val[j]);
    key_out[p] = k;
    val_out[p] = acc;
  }
};

template <class V, class Op>
int reduce_by_key(const uint32_t *key, const V *val, size_t n, uint32_t *key_out, V *val_out,
                  int64_t *d_n_out, Op op, Scratch &S, hipStream_t s) {
  return compact(n, RunHead{key}, FoldRun<V, Op>{key, val, n, key_out, val_out, op}, d_n_out, S,
                 s);
}

}  // namespace prim
}  // namespace inet

#endif
