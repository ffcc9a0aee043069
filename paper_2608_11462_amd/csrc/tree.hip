// Geometry normalisation and the uniform quadtree (paper Sec. 2.1 step 1,
// "tree creation"; normalisation per eq. M_rho and the domains of Sec. 2.2).
//
// Nodes are normalised to xi = (x - c) * rho, quantised to a 2^L x 2^L grid
// over [-h, h]^2 and sorted stably by the row-major leaf key, so that the
// three leaves of one grid row that neighbour a leaf occupy one contiguous
// range of the tree order.
#include "phs_internal.h"

// Normalisation and quantisation must round exactly as written (they decide
// integer cell indices that are compared with an independent reference).
#pragma clang fp contract(off)

namespace phs {

void scan_exclusive(int32_t *data, int64_t count, int32_t *ws, hipStream_t s);
int64_t scan_ws_ints(int64_t count);

namespace {

constexpr int kBlock = 256;

__global__ void k_minmax_partial(const double *__restrict__ xy, int64_t n,
                                 double *__restrict__ part) {
  __shared__ double s[4][kBlock];
  double mnx = INFINITY, mny = INFINITY, mxx = -INFINITY, mxy = -INFINITY;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    double a = xy[2 * i], b = xy[2 * i + 1];
    mnx = fmin(mnx, a);
    mxx = fmax(mxx, a);
    mny = fmin(mny, b);
    mxy = fmax(mxy, b);
  }
  s[0][threadIdx.x] = mnx;
  s[1][threadIdx.x] = mny;
  s[2][threadIdx.x] = mxx;
  s[3][threadIdx.x] = mxy;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + w]);
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) part[blockIdx.x * 4 + threadIdx.x] = s[threadIdx.x][0];
}

// min and max are exact in any order, so the tree over threads gives the
// result of a sequential pass.
__global__ void k_minmax_final(const double *__restrict__ part, int nb,
                               double *__restrict__ out) {
  __shared__ double s[4][kBlock];
  double r[4] = {INFINITY, INFINITY, -INFINITY, -INFINITY};
  for (int b = threadIdx.x; b < nb; b += kBlock) {
    r[0] = fmin(r[0], part[4 * b + 0]);
    r[1] = fmin(r[1], part[4 * b + 1]);
    r[2] = fmax(r[2], part[4 * b + 2]);
    r[3] = fmax(r[3], part[4 * b + 3]);
  }
  for (int t = 0; t < 4; ++t) s[t][threadIdx.x] = r[t];
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
      s[1][threadIdx.x] = fmin(s[1][threadIdx.x], s[1][threadIdx.x + w]);
      s[2][threadIdx.x] = fmax(s[2][threadIdx.x], s[2][threadIdx.x + w]);
      s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x < 4) out[threadIdx.x] = s[threadIdx.x][0];
}

// Quantise one normalised coordinate to a grid cell index in [0, G).
// (xi + h) is the only rounded step: G / (2h) is a power of two.
__device__ __forceinline__ int cell_of(double xi, double h, double scale, int G) {
  double u = (xi + h) * scale;
  int q = (int)floor(u);
  q = q < 0 ? 0 : q;
  return q >= G ? G - 1 : q;
}

__global__ void k_leaf_keys(const double *__restrict__ xy, int64_t n, double cx,
                            double cy, double rho, double h, int L,
                            uint32_t *__restrict__ keys,
                            int32_t *__restrict__ idx) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int G = 1 << L;
  const double scale = (double)G / (2.0 * h);
  double xi = (xy[2 * i] - cx) * rho;
  double yi = (xy[2 * i + 1] - cy) * rho;
  int ix = cell_of(xi, h, scale, G), iy = cell_of(yi, h, scale, G);
  keys[i] = (uint32_t)iy * (uint32_t)G + (uint32_t)ix;
  idx[i] = (int32_t)i;
}

// ---------------------------------------------------------------- radix sort
constexpr int kRadixBits = 8;
constexpr int kBuckets = 1 << kRadixBits;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;

constexpr int kWaves = kBlock / 64;
constexpr int kWaveItems = kTile / kWaves;  // each wave takes a contiguous chunk

// Lanes of the wave holding the same digit as this lane (8 ballots, one per
// digit bit), restricted to the valid lanes.
__device__ __forceinline__ uint64_t digit_peers(int digit, bool valid) {
  uint64_t mask = __ballot(valid);
#pragma unroll
  for (int b = 0; b < kRadixBits; ++b) {
    const bool bit = (digit >> b) & 1;
    const uint64_t bb = __ballot(valid && bit);
    mask &= bit ? bb : ~bb;
  }
  return mask;
}

// Digit histogram of each tile: hist[digit * nblocks + tile].
template <class K>
__global__ void k_radix_hist(const K *__restrict__ keys, int64_t n, int shift,
                             int nblocks, int32_t *__restrict__ hist) {
  __shared__ int cnt[kBuckets];
  cnt[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + it * kBlock + threadIdx.x;
    if (i < n) atomicAdd(&cnt[(int)((keys[i] >> shift) & (kBuckets - 1))], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter of one tile by the digit at `shift`.  The tile is first
// counting-sorted in LDS (wave w holds keys [w * kWaveItems, (w+1) * kWaveItems)
// of the tile, so a key's rank among equal digits is the count in earlier
// waves plus the count earlier in its own wave), then written out in that
// order, so neighbouring lanes store neighbouring addresses of a bucket.
// offs[digit * nblocks + tile] is the exclusive scan of the histograms.
template <class K>
__global__ __launch_bounds__(kBlock) void k_radix_scatter(
    const K *__restrict__ keys, const int32_t *__restrict__ vals, int64_t n, int shift,
    int nblocks, const int32_t *__restrict__ offs, K *__restrict__ okeys,
    int32_t *__restrict__ ovals) {
  __shared__ int wcnt[kWaves][kBuckets];  // running counts, then wave offsets
  __shared__ int lstart[kBuckets];        // first tile slot of each digit
  __shared__ int goff[kBuckets];          // output index of that slot
  __shared__ int wsum[kWaves];
  __shared__ K skey[kTile];
  __shared__ int32_t sval[kTile];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int w = 0; w < kWaves; ++w) wcnt[w][tid] = 0;
  goff[tid] = offs[tid * nblocks + blockIdx.x];
  __syncthreads();
  const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t tile0 = (int64_t)blockIdx.x * kTile;
  const int64_t base = tile0 + wave * kWaveItems;
  K key[kItems];
  int32_t val[kItems];
  int rank[kItems];
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int64_t i = base + it * 64 + lane;
    const bool valid = i < n;
    key[it] = valid ? keys[i] : K(0);
    val[it] = valid ? vals[i] : 0;
  }
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const bool valid = base + it * 64 + lane < n;
    const int digit = (int)((key[it] >> shift) & (kBuckets - 1));
    const uint64_t peers = digit_peers(digit, valid);
    const int before = valid ? wcnt[wave][digit] : 0;
    rank[it] = before + __popcll(peers & lt_mask);
    // LDS operations of one wave complete in order: every lane has read the
    // count before its leader stores the new one.
    if (valid && (peers & lt_mask) == 0) wcnt[wave][digit] = before + __popcll(peers);
  }
  __syncthreads();
  int tot = 0;
  for (int w = 0; w < kWaves; ++w) {
    const int c = wcnt[w][tid];
    wcnt[w][tid] = tot;
    tot += c;
  }
  int incl = tot;  // inclusive scan over digits: within the wave, then across waves
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int add = 0;
  for (int w = 0; w < wave; ++w) add += wsum[w];
  lstart[tid] = add + incl - tot;
  __syncthreads();
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    if (base + it * 64 + lane < n) {
      const int digit = (int)((key[it] >> shift) & (kBuckets - 1));
      const int pos = lstart[digit] + wcnt[wave][digit] + rank[it];
      skey[pos] = key[it];
      sval[pos] = val[it];
    }
  }
  __syncthreads();
  const int64_t rem = n - tile0;
  const int cnt = rem < kTile ? (int)rem : kTile;
#pragma unroll
  for (int it = 0; it < kItems; ++it) {
    const int p = it * kBlock + tid;
    if (p < cnt) {
      const K k = skey[p];
      const int digit = (int)((k >> shift) & (kBuckets - 1));
      const int64_t o = (int64_t)goff[digit] + (p - lstart[digit]);
      okeys[o] = k;
      ovals[o] = sval[p];
    }
  }
}

// With `in_tmp` given, an odd number of passes leaves the result in
// (ktmp, vtmp) and *in_tmp says so; otherwise it is copied back.
template <class K>
void radix_sort(K *keys, int32_t *vals, int64_t n, int bits, K *ktmp,
                int32_t *vtmp, int32_t *scratch, hipStream_t s, bool *in_tmp) {
  if (in_tmp) *in_tmp = false;
  if (n <= 1) return;
  int nblocks = (int)((n + kTile - 1) / kTile);
  int32_t *hist = scratch;
  int32_t *ws = scratch + (int64_t)kBuckets * nblocks;
  int passes = (bits + kRadixBits - 1) / kRadixBits;
  K *src_k = keys, *dst_k = ktmp;
  int32_t *src_v = vals, *dst_v = vtmp;
  for (int p = 0; p < passes; ++p) {
    int shift = p * kRadixBits;
    PHS_LAUNCH("radix_hist", s,
               k_radix_hist<K><<<nblocks, kBlock, 0, s>>>(src_k, n, shift,
                                                           nblocks, hist));
    scan_exclusive(hist, (int64_t)kBuckets * nblocks, ws, s);
    PHS_LAUNCH("radix_scatter", s,
               k_radix_scatter<K><<<nblocks, kBlock, 0, s>>>(
                   src_k, src_v, n, shift, nblocks, hist, dst_k, dst_v));
    std::swap(src_k, dst_k);
    std::swap(src_v, dst_v);
  }
  if (src_k != keys && in_tmp) {
    *in_tmp = true;
  } else if (src_k != keys) {
    PHS_HIP(hipMemcpyAsync(keys, src_k, n * sizeof(K), hipMemcpyDeviceToDevice, s));
    PHS_HIP(hipMemcpyAsync(vals, src_v, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
}

__global__ void k_leaf_ranges(const uint32_t *__restrict__ keys, int64_t n,
                              int nleaves, int32_t *__restrict__ start) {
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c > nleaves) return;
  // lower_bound of c in keys
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < (uint32_t)c) lo = mid + 1;
    else hi = mid;
  }
  start[c] = (int32_t)lo;
}

__global__ void k_tree_points(const double *__restrict__ xy,
                              const int32_t *__restrict__ order,
                              const uint32_t *__restrict__ keys, int64_t n,
                              double cx, double cy, double rho, double h, int L,
                              double *__restrict__ x, double *__restrict__ y,
                              float *__restrict__ ux, float *__restrict__ uy,
                              double2 *__restrict__ xy2, int32_t *__restrict__ leafkey,
                              int32_t *__restrict__ inv) {
  int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  int u = order[i];
  double xi = (xy[2 * (int64_t)u] - cx) * rho;
  double yi = (xy[2 * (int64_t)u + 1] - cy) * rho;
  x[i] = xi;
  y[i] = yi;
  xy2[i] = make_double2(xi, yi);
  const int G = 1 << L;
  uint32_t key = keys[i];
  int ix = (int)(key % (uint32_t)G), iy = (int)(key / (uint32_t)G);
  double w = 2.0 * h / G;
  double ccx = -h + (ix + 0.5) * w, ccy = -h + (iy + 0.5) * w;
  ux[i] = (float)(xi - ccx);
  uy[i] = (float)(yi - ccy);
  leafkey[i] = (int32_t)key;
  inv[u] = (int32_t)i;
}

// Flags coincident nodes: within one leaf (coincident nodes share a leaf).
__global__ void k_dup(const double *__restrict__ x, const double *__restrict__ y,
                      const int32_t *__restrict__ start, int nleaves,
                      int32_t *__restrict__ flag) {
  int leaf = blockIdx.x;
  if (leaf >= nleaves) return;
  int b = start[leaf], e = start[leaf + 1];
  for (int i = b + threadIdx.x; i < e; i += blockDim.x) {
    double xi = x[i], yi = y[i];
    for (int j = i + 1; j < e; ++j)
      if (x[j] == xi && y[j] == yi) flag[0] = 1;
  }
}

}  // namespace

// Exclusive scan of int32 in place, blocks of 4*kBlock elements.
constexpr int kScanTile = 4 * kBlock;

__device__ int block_exclusive_scan(int v, int *sh_waves, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int x = v;
  for (int o = 1; o < 64; o <<= 1) {
    int y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == 63) sh_waves[wave] = x;
  __syncthreads();
  int wbase = 0, tot = 0;
  for (int w = 0; w < kBlock / 64; ++w) {
    if (w < wave) wbase += sh_waves[w];
    tot += sh_waves[w];
  }
  *total = tot;
  __syncthreads();
  return wbase + x - v;
}

__global__ void k_scan_block(int32_t *__restrict__ data, int64_t count,
                             int32_t *__restrict__ sums) {
  __shared__ int sh[kBlock / 64];
  int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  int v[4];
  int loc = 0;
  for (int t = 0; t < 4; ++t) {
    v[t] = (base + t < count) ? data[base + t] : 0;
    loc += v[t];
  }
  int tot;
  int ex = block_exclusive_scan(loc, sh, &tot);
  for (int t = 0; t < 4; ++t) {
    if (base + t < count) data[base + t] = ex;
    ex += v[t];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void k_scan_add(int32_t *__restrict__ data, int64_t count,
                           const int32_t *__restrict__ sums) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + 4 * threadIdx.x;
  int add = sums[blockIdx.x];
  for (int t = 0; t < 4; ++t)
    if (base + t < count) data[base + t] += add;
}

void scan_exclusive(int32_t *data, int64_t count, int32_t *ws, hipStream_t s) {
  int64_t nb = (count + kScanTile - 1) / kScanTile;
  PHS_LAUNCH("scan", s, k_scan_block<<<nb, kBlock, 0, s>>>(data, count, ws));
  if (nb > 1) {
    scan_exclusive(ws, nb, ws + nb, s);
    PHS_LAUNCH("scan", s, k_scan_add<<<nb, kBlock, 0, s>>>(data, count, ws));
  }
}

int64_t scan_ws_ints(int64_t count) {
  int64_t tot = 0;
  while (count > 1) {
    count = (count + kScanTile - 1) / kScanTile;
    tot += count;
  }
  return tot + 1;
}


void minmax_xy(const double *xy, int64_t n, double *out4, double *partials,
               int nblocks, hipStream_t s) {
  PHS_LAUNCH("minmax", s,
             k_minmax_partial<<<nblocks, kBlock, 0, s>>>(xy, n, partials));
  PHS_LAUNCH("minmax", s, k_minmax_final<<<1, kBlock, 0, s>>>(partials, nblocks, out4));
}

void leaf_keys(const double *xy, int64_t n, double cx, double cy, double rho,
               double h, int L, uint32_t *keys, int32_t *idx, hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("leaf_keys", s,
             k_leaf_keys<<<nb, kBlock, 0, s>>>(xy, n, cx, cy, rho, h, L, keys, idx));
}

size_t radix_sort_scratch_ints(int64_t n) {
  int64_t nblocks = (n + kTile - 1) / kTile;
  return (size_t)(kBuckets * nblocks + scan_ws_ints(kBuckets * nblocks) + 16);
}

void radix_sort_u32(uint32_t *keys, int32_t *vals, int64_t n, int bits,
                    uint32_t *ktmp, int32_t *vtmp, int32_t *scratch,
                    hipStream_t s, bool *in_tmp) {
  radix_sort<uint32_t>(keys, vals, n, bits, ktmp, vtmp, scratch, s, in_tmp);
}

void radix_sort_u64(uint64_t *keys, int32_t *vals, int64_t n, int bits,
                    uint64_t *ktmp, int32_t *vtmp, int32_t *scratch,
                    hipStream_t s) {
  radix_sort<uint64_t>(keys, vals, n, bits, ktmp, vtmp, scratch, s, nullptr);
}

void leaf_ranges(const uint32_t *sorted_keys, int64_t n, int nleaves,
                 int32_t *leaf_start, hipStream_t s) {
  int nb = (nleaves + 1 + kBlock - 1) / kBlock;
  PHS_LAUNCH("leaf_ranges", s,
             k_leaf_ranges<<<nb, kBlock, 0, s>>>(sorted_keys, n, nleaves, leaf_start));
}

void build_tree_points(const double *xy, const int32_t *order,
                       const uint32_t *keys_sorted, int64_t n, double cx,
                       double cy, double rho, double h, int L, double *x,
                       double *y, float *ux, float *uy, double2 *xy2, int32_t *leafkey,
                       int32_t *inv_order, hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("tree_points", s,
             k_tree_points<<<nb, kBlock, 0, s>>>(xy, order, keys_sorted, n, cx, cy,
                                                 rho, h, L, x, y, ux, uy, xy2, leafkey,
                                                 inv_order));
}

void count_duplicates(const double *x, const double *y, const int32_t *leaf_start,
                      int nleaves, int32_t *flag, hipStream_t s) {
  PHS_LAUNCH("dup_check", s, k_dup<<<nleaves, 64, 0, s>>>(x, y, leaf_start, nleaves, flag));
}

}  // namespace phs
