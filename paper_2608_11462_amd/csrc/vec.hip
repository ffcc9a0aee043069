// Plan-time vector kernels of the polynomial block (paper eq. phs_linsys_solve
// and the O(nS) complement projector, Sec. 2): the block P of the tree-ordered
// nodes, its Gram matrix by deterministic multi-dot reductions, and the
// column transform of CholeskyQR.  The PCG's own vector kernels run on the
// batched engine.
//
// Reductions are two-stage with a grid size that depends only on n, so every
// result is bitwise reproducible run to run.
#include "phs_internal.h"

namespace phs {

namespace {

constexpr int kBlock = 256;
constexpr int kMaxDots = 32;

struct DotArgs {
  const double *a[kMaxDots];
  const double *b[kMaxDots];
};

inline int grid_for(int64_t n) {
  int64_t nb = (n + kBlock * 4 - 1) / (kBlock * 4);
  if (nb > 1024) nb = 1024;
  if (nb < 1) nb = 1;
  return (int)nb;
}

__device__ __forceinline__ double block_sum(double v, double *sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) sh[wave] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kBlock / 64; ++w) t += sh[w];
  __syncthreads();
  return t;  // valid in thread 0
}

template <int ND>
__global__ void k_multi_dot(DotArgs args, int nd, int64_t n,
                            double *__restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double acc[ND];
  for (int t = 0; t < ND; ++t) acc[t] = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    for (int t = 0; t < ND; ++t)
      if (t < nd) acc[t] += args.a[t][i] * args.b[t][i];
  }
  for (int t = 0; t < ND; ++t) {
    if (t >= nd) break;
    double s = block_sum(acc[t], sh);
    if (threadIdx.x == 0) part[t * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void k_reduce_final(const double *__restrict__ part, int nb, int nd,
                               double *__restrict__ out) {
  __shared__ double sh[kBlock / 64];
  for (int t = 0; t < nd; ++t) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) v += part[t * nb + b];
    double s = block_sum(v, sh);
    if (threadIdx.x == 0) out[t] = s;
  }
}

__global__ void k_poly_block(const double *__restrict__ x, const double *__restrict__ y,
                             int64_t n, int d, double *__restrict__ B) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  double px[8], py[8];
  px[0] = py[0] = 1.0;
  for (int e = 1; e <= d; ++e) {
    px[e] = px[e - 1] * x[i];
    py[e] = py[e - 1] * y[i];
  }
  int col = 0;
  for (int t = 0; t <= d; ++t)
    for (int a = t; a >= 0; --a) B[(int64_t)col++ * n + i] = px[a] * py[t - a];
}

__global__ void k_apply_rinv(double *__restrict__ B, int64_t n, int S,
                             const double *__restrict__ Rinv) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  double b[28], o[28];
  for (int j = 0; j < S; ++j) b[j] = B[(int64_t)j * n + i];
  for (int j = 0; j < S; ++j) {
    double s = 0.0;
    for (int l = 0; l <= j; ++l) s += b[l] * Rinv[l * S + j];
    o[j] = s;
  }
  for (int j = 0; j < S; ++j) B[(int64_t)j * n + i] = o[j];
}

}  // namespace

int dot_blocks(int64_t n) { return grid_for(n); }

void poly_block_tree(const double *x, const double *y, int64_t n, int d, double *B,
                     hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("poly_block", s, k_poly_block<<<nb, kBlock, 0, s>>>(x, y, n, d, B));
}

// sum_i a_t[i] b_t[i] for t < nd into out (device), two-stage
static void multi_dot(const double *const *a, const double *const *b, int nd, int64_t n,
                      double *partials, double *out, hipStream_t s) {
  PHS_REQUIRE(nd >= 1 && nd <= kMaxDots, PHS_ERR_INVALID_ARGUMENT, "multi_dot: bad count");
  DotArgs args;
  for (int t = 0; t < nd; ++t) {
    args.a[t] = a[t];
    args.b[t] = b[t];
  }
  int nb = grid_for(n);
  if (nd <= 4)
    PHS_LAUNCH("dot", s, k_multi_dot<4><<<nb, kBlock, 0, s>>>(args, nd, n, partials));
  else if (nd <= 8)
    PHS_LAUNCH("dot", s, k_multi_dot<8><<<nb, kBlock, 0, s>>>(args, nd, n, partials));
  else
    PHS_LAUNCH("dot", s, k_multi_dot<kMaxDots><<<nb, kBlock, 0, s>>>(args, nd, n, partials));
  PHS_LAUNCH("dot_final", s, k_reduce_final<<<1, kBlock, 0, s>>>(partials, nb, nd, out));
}

void gram(const double *B, int64_t n, int S, double *partials, double *out, hipStream_t s) {
  // out[a*S+b] for a <= b, computed in chunks of kMaxDots pairs
  std::vector<std::pair<int, int>> pairs;
  for (int a = 0; a < S; ++a)
    for (int b = a; b < S; ++b) pairs.push_back({a, b});
  for (size_t off = 0; off < pairs.size(); off += kMaxDots) {
    int nd = (int)std::min<size_t>(kMaxDots, pairs.size() - off);
    const double *pa[kMaxDots], *pb[kMaxDots];
    for (int t = 0; t < nd; ++t) {
      pa[t] = B + (int64_t)pairs[off + t].first * n;
      pb[t] = B + (int64_t)pairs[off + t].second * n;
    }
    multi_dot(pa, pb, nd, n, partials, out + off, s);
  }
}

void apply_rinv(double *B, int64_t n, int S, const double *Rinv, hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("apply_rinv", s, k_apply_rinv<<<nb, kBlock, 0, s>>>(B, n, S, Rinv));
}

}  // namespace phs
