// Vector kernels of the projected PCG (paper eq. phs_linsys_solve and the
// O(nS) application of the complement projector, Sec. 2): permutations, the
// polynomial block, deterministic multi-dot reductions, the projector
// Pi v = v - Q (Q^T v), and the fused PCG recurrences.
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

__global__ void k_gather(const double *__restrict__ src, const int32_t *__restrict__ order,
                         int64_t n, double *__restrict__ dst) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) dst[i] = src[order[i]];
}

__global__ void k_scatter(const double *__restrict__ src, const int32_t *__restrict__ order,
                          int64_t n, double *__restrict__ dst) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) dst[order[i]] = src[i];
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

__global__ void k_sub_Qc(double *__restrict__ v, const double *__restrict__ Q,
                         int64_t n, int S, const double *__restrict__ c) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int j = 0; j < S; ++j) s += Q[(int64_t)j * n + i] * c[j];
  v[i] -= s;
}

__global__ void k_axpby(double *__restrict__ y, const double *__restrict__ x, double a,
                        double b, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

__global__ void k_scale_copy(double *__restrict__ d, const double *__restrict__ s, double a,
                             int64_t n) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) d[i] = a * s[i];
}

__global__ void k_fill(double *__restrict__ v, double a, int64_t n) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  if (i < n) v[i] = a;
}

// w += alpha p, r -= alpha q with alpha = num/den read from device memory,
// and per-block partial sums of r.r.
__global__ void k_pcg_wr(double *__restrict__ w, double *__restrict__ r,
                         const double *__restrict__ p, const double *__restrict__ q,
                         const double *__restrict__ num, const double *__restrict__ den,
                         int64_t n, double *__restrict__ part) {
  __shared__ double sh[kBlock / 64];
  const double alpha = num[0] / den[0];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kBlock) {
    w[i] += alpha * p[i];
    double ri = r[i] - alpha * q[i];
    r[i] = ri;
    acc += ri * ri;
  }
  double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_pcg_p(double *__restrict__ p, const double *__restrict__ z,
                        const double *__restrict__ num, const double *__restrict__ den,
                        int64_t n) {
  int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x;
  const double beta = num[0] / den[0];
  if (i < n) p[i] = z[i] + beta * p[i];
}

}  // namespace

int dot_blocks(int64_t n) { return grid_for(n); }

void gather_cols(const double *src_user, const int32_t *order, int64_t n, double *dst_tree,
                 hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("gather", s, k_gather<<<nb, kBlock, 0, s>>>(src_user, order, n, dst_tree));
}

void scatter_cols(const double *src_tree, const int32_t *order, int64_t n, double *dst_user,
                  hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("scatter", s, k_scatter<<<nb, kBlock, 0, s>>>(src_tree, order, n, dst_user));
}

void poly_block_tree(const double *x, const double *y, int64_t n, int d, double *B,
                     hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("poly_block", s, k_poly_block<<<nb, kBlock, 0, s>>>(x, y, n, d, B));
}

void multi_dot(const double *const *a, const double *const *b, int nd, int64_t n,
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

void project(double *v, const double *Q, int64_t n, int S, double *partials, double *scal,
             hipStream_t s) {
  const double *pa[kMaxDots], *pb[kMaxDots];
  for (int j = 0; j < S; ++j) {
    pa[j] = Q + (int64_t)j * n;
    pb[j] = v;
  }
  multi_dot(pa, pb, S, n, partials, scal, s);
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("project", s, k_sub_Qc<<<nb, kBlock, 0, s>>>(v, Q, n, S, scal));
}

void axpby(double *y, const double *x, double a, double b, int64_t n, hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("axpby", s, k_axpby<<<nb, kBlock, 0, s>>>(y, x, a, b, n));
}

void scale_copy(double *dst, const double *src, double a, int64_t n, hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("scale_copy", s, k_scale_copy<<<nb, kBlock, 0, s>>>(dst, src, a, n));
}

void fill(double *v, double a, int64_t n, hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("fill", s, k_fill<<<nb, kBlock, 0, s>>>(v, a, n));
}

void copy(double *dst, const double *src, int64_t n, hipStream_t s) {
  PHS_HIP(hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
}

// num/den are scal[0]/scal[1] for the (w, r) update; the caller supplies
// pointers to the slots it uses.
void pcg_update_wr(double *w, double *r, const double *p, const double *q,
                   const double *scal, int64_t n, double *partials, double *out_rr,
                   hipStream_t s) {
  int nb = grid_for(n);
  PHS_LAUNCH("pcg_wr", s,
             k_pcg_wr<<<nb, kBlock, 0, s>>>(w, r, p, q, scal, scal + 1, n, partials));
  PHS_LAUNCH("dot_final", s, k_reduce_final<<<1, kBlock, 0, s>>>(partials, nb, 1, out_rr));
}

void pcg_update_p(double *p, const double *z, const double *scal, int64_t n,
                  hipStream_t s) {
  int64_t nb = (n + kBlock - 1) / kBlock;
  PHS_LAUNCH("pcg_p", s, k_pcg_p<<<nb, kBlock, 0, s>>>(p, z, scal, scal + 1, n));
}

}  // namespace phs
