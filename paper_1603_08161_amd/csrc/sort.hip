// Stable key/value sort and integer exclusive prefix sums on the device: the
// binning of constraint rows by lattice cell (the rows of a cell become one
// contiguous segment, Sec. 7.1's per-cell B^T B blocks), the slots of the
// nodes that carry data blocks, and the output offsets of marching cubes.
//
// Sort: least-significant-digit radix sort over 8-bit digits.  Each pass
// counts the digits of every block of 1024 rows, scans the counts in
// digit-major order (all blocks of digit 0, then digit 1, ...) into each
// (digit, block)'s first output position, and scatters the block's rows.
// Inside a block the rows form 16 chunks of 64, one per wave at a time; the
// lanes of a chunk find the lanes holding the same digit with one ballot per
// digit bit, which gives each row its rank among the equal digits before it
// in the chunk, and a per-digit prefix over the chunks orders the chunks.
// Every row thus keeps the input order among equal digits, so each pass is
// stable and the sort orders by key with ties in input order.
//
// Scan: block sums of 1024 elements, a one-workgroup exclusive scan of the
// block sums, then each block's own exclusive scan offset by its sum.
//
// Integer arithmetic only: both are exact, and the results do not depend on
// the order in which the hardware schedules the workgroups.
#include "vd_device.h"
#include "vd_kernels.h"

namespace vd {

namespace {

constexpr int kThreads = 256;                 // 4 waves
constexpr int kWaves = kThreads / kWave;
constexpr int kSortTile = 1024;               // rows per block and pass
constexpr int kChunks = kSortTile / kWave;    // 16 chunks of 64 rows
constexpr int kChunksPerWave = kChunks / kWaves;
constexpr int kDigitBits = 8;
constexpr int kBuckets = 1 << kDigitBits;     // 256 = one per thread
constexpr int kScanTile = 1024;               // elements per scan block
constexpr int kPerThread = kScanTile / kThreads;
static_assert(kBuckets == kThreads, "one digit bucket per thread");

inline int ceil_div(int64_t n, int d) { return (int)((n + d - 1) / d); }
inline size_t aligned(size_t bytes) { return (bytes + 255) & ~(size_t)255; }

// Exclusive prefix of v over the block's threads in thread order; *total
// (shared by all threads) receives the block's sum.
__device__ __forceinline__ int block_exclusive(int v, int* total) {
  __shared__ int wave_sum[kWaves];
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  int inc = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int t = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += t;
  }
  if (lane == kWave - 1) wave_sum[wv] = inc;
  __syncthreads();
  int before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) {
    if (w < wv) before += wave_sum[w];
    all += wave_sum[w];
  }
  __syncthreads();  // wave_sum may be reused by the next call
  *total = all;
  return before + inc - v;
}

// sums[b] = sum of in[b * kScanTile .. (b + 1) * kScanTile) (within n).
__global__ __launch_bounds__(kThreads) void k_scan_block_sums(const int* __restrict__ in,
                                                              int64_t n, int* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kPerThread;
  int v = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k)
    if (base + k < n) v += in[base + k];
  int total;
  (void)block_exclusive(v, &total);
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// In-place exclusive scan of the nb block sums (one workgroup, in order).
__global__ __launch_bounds__(kThreads) void k_scan_sums(int* sums, int nb) {
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += kScanTile) {
    const int base = c0 + threadIdx.x * kPerThread;
    int v[kPerThread], s = 0;
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      v[k] = base + k < nb ? sums[base + k] : 0;
      s += v[k];
    }
    int total;
    int run = carry + block_exclusive(s, &total);
#pragma unroll
    for (int k = 0; k < kPerThread; ++k) {
      if (base + k < nb) sums[base + k] = run;
      run += v[k];
    }
    carry += total;
  }
}

// out = exclusive prefix sum of in, given the scanned block sums.
__global__ __launch_bounds__(kThreads) void k_scan_apply(const int* __restrict__ in, int64_t n,
                                                         const int* __restrict__ sums,
                                                         int* __restrict__ out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kPerThread;
  int v[kPerThread], s = 0;
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    v[k] = base + k < n ? in[base + k] : 0;
    s += v[k];
  }
  int total;
  int run = sums[blockIdx.x] + block_exclusive(s, &total);
#pragma unroll
  for (int k = 0; k < kPerThread; ++k) {
    if (base + k < n) out[base + k] = run;
    run += v[k];
  }
}

// hist[d * nblocks + b] = rows of block b whose digit (key >> shift) & 255 is d.
__global__ __launch_bounds__(kThreads) void k_digit_hist(const unsigned* __restrict__ keys,
                                                         int n, int shift, int nblocks,
                                                         int* __restrict__ hist) {
  __shared__ int h[kBuckets];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortTile;
  for (int j = threadIdx.x; j < kSortTile; j += kThreads) {
    const int r = base + j;
    if (r < n) atomicAdd(&h[(keys[r] >> shift) & (kBuckets - 1)], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of block b's rows to offs[digit * nblocks + b] + (rows of
// the same digit before them in the block).
__global__ __launch_bounds__(kThreads) void k_digit_scatter(
    const unsigned* __restrict__ kin, const int* __restrict__ vin, unsigned* __restrict__ kout,
    int* __restrict__ vout, int n, int shift, int nblocks, const int* __restrict__ offs) {
  __shared__ int cnt[kChunks][kBuckets];  // rows per (chunk, digit), then their prefix
  for (int i = threadIdx.x; i < kChunks * kBuckets; i += kThreads) (&cnt[0][0])[i] = 0;
  __syncthreads();
  const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
  const unsigned long long below = (1ull << lane) - 1ull;
  const int base = blockIdx.x * kSortTile;
  unsigned key[kChunksPerWave];
  int val[kChunksPerWave], dig[kChunksPerWave], rank[kChunksPerWave];
  bool ok[kChunksPerWave];
#pragma unroll
  for (int q = 0; q < kChunksPerWave; ++q) {
    const int c = wv + q * kWaves;  // chunks in row order, dealt to the waves
    const int r = base + c * kWave + lane;
    ok[q] = r < n;
    key[q] = ok[q] ? kin[r] : 0u;
    val[q] = ok[q] ? vin[r] : 0;
    const int d = (int)((key[q] >> shift) & (kBuckets - 1));
    dig[q] = d;
    // lanes of the chunk with the same digit: agree on every digit bit
    unsigned long long peers = __ballot(ok[q]);
#pragma unroll
    for (int bit = 0; bit < kDigitBits; ++bit) {
      const bool set = ((d >> bit) & 1) != 0;
      const unsigned long long m = __ballot(ok[q] && set);
      peers &= set ? m : ~m;
    }
    rank[q] = __popcll(peers & below);
    if (ok[q] && rank[q] == 0) cnt[c][d] = __popcll(peers);
  }
  __syncthreads();
  {
    const int d = threadIdx.x;  // thread d: exclusive prefix of digit d over the chunks
    int run = 0;
    for (int c = 0; c < kChunks; ++c) {
      const int t = cnt[c][d];
      cnt[c][d] = run;
      run += t;
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kChunksPerWave; ++q) {
    if (!ok[q]) continue;
    const int c = wv + q * kWaves;
    const int pos = offs[dig[q] * nblocks + blockIdx.x] + cnt[c][dig[q]] + rank[q];
    kout[pos] = key[q];
    vout[pos] = val[q];
  }
}

// Scratch of an n-row sort: digit counts and their scan, the scan's block
// sums, and the key/value ping-pong buffers.
struct SortScratch {
  int *hist, *offs, *sums;
  unsigned* ktmp;
  int* vtmp;
};

size_t sort_layout(int n, char* base, SortScratch* sc) {
  const int nblocks = ceil_div(n, kSortTile);
  const int64_t H = (int64_t)kBuckets * nblocks;
  const size_t sizes[5] = {aligned(4 * (size_t)H), aligned(4 * (size_t)H),
                           aligned(4 * (size_t)ceil_div(H, kScanTile)), aligned(4 * (size_t)n),
                           aligned(4 * (size_t)n)};
  if (base && sc) {
    char* p = base;
    sc->hist = (int*)p; p += sizes[0];
    sc->offs = (int*)p; p += sizes[1];
    sc->sums = (int*)p; p += sizes[2];
    sc->ktmp = (unsigned*)p; p += sizes[3];
    sc->vtmp = (int*)p;
  }
  return sizes[0] + sizes[1] + sizes[2] + sizes[3] + sizes[4];
}

hipError_t scan_with(int* sums, const int* in, int* out, int64_t n, hipStream_t s) {
  const int nb = ceil_div(n, kScanTile);
  k_scan_block_sums<<<nb, kThreads, 0, s>>>(in, n, sums);
  k_scan_sums<<<1, kThreads, 0, s>>>(sums, nb);
  k_scan_apply<<<nb, kThreads, 0, s>>>(in, n, sums, out);
  return hipGetLastError();
}

}  // namespace

size_t sort_temp_bytes(int n) { return n > 0 ? sort_layout(n, nullptr, nullptr) : 0; }

hipError_t sort_pairs(void* temp, size_t bytes, const unsigned* kin, unsigned* kout,
                      const int* vin, int* vout, int n, int end_bit, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n < 0 || end_bit < 0 || end_bit > 32 || !temp || bytes < sort_temp_bytes(n))
    return hipErrorInvalidValue;
  const int passes = (end_bit + kDigitBits - 1) / kDigitBits;
  if (passes == 0) {  // every key is 0: the order is the input order
    hipError_t e = hipMemcpyAsync(kout, kin, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(vout, vin, 4 * (size_t)n, hipMemcpyDeviceToDevice, s);
    return e;
  }
  SortScratch sc;
  sort_layout(n, (char*)temp, &sc);
  const int nblocks = ceil_div(n, kSortTile);
  const unsigned* ksrc = kin;
  const int* vsrc = vin;
  for (int p = 0; p < passes; ++p) {
    // the last pass lands in the caller's output, the ones before alternate
    const bool to_out = ((passes - p) & 1) == 1;
    unsigned* kdst = to_out ? kout : sc.ktmp;
    int* vdst = to_out ? vout : sc.vtmp;
    const int shift = p * kDigitBits;
    k_digit_hist<<<nblocks, kThreads, 0, s>>>(ksrc, n, shift, nblocks, sc.hist);
    hipError_t e = scan_with(sc.sums, sc.hist, sc.offs, (int64_t)kBuckets * nblocks, s);
    if (e != hipSuccess) return e;
    k_digit_scatter<<<nblocks, kThreads, 0, s>>>(ksrc, vsrc, kdst, vdst, n, shift, nblocks,
                                                 sc.offs);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ksrc = kdst;
    vsrc = vdst;
  }
  return hipSuccess;
}

size_t scan_temp_bytes(int n) { return aligned(4 * (size_t)ceil_div(n > 0 ? n : 1, kScanTile)); }

hipError_t exclusive_scan(void* temp, size_t bytes, const int* in, int* out, int n,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (n < 0 || !temp || bytes < scan_temp_bytes(n)) return hipErrorInvalidValue;
  return scan_with((int*)temp, in, out, n, s);
}

}  // namespace vd
