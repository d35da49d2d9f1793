// lc_fourier.hip -- Fourier-mode improved estimators of one sweep's loops
// (the second-moment estimators of the correlation length and the gap,
// which the paper cites for its S = 1 results, Sec. 5).
//
// Along a loop the staggered spin (-1)^j S^z_j is one value +-1/2, so
// S^z at momentum pi + d and Matsubara frequency w is a sum over loops of
// +-1/2 times Q_c(d, w) = sum over the loop's vertical segments (site j,
// from tau_a to tau_b) of e^{i d j} int e^{i w tau} dtau, and
// chi(pi + d, w) = <sum_c |Q_c|^2> / (4 beta L).
//
// Each segment's integral splits over its two end nodes, so every node adds
// a term of its own to its loop's sums: an operator node at time t joins the
// two segments of its two subspins x, y (sites jx, jy) -- its lower node
// ends them (+), its upper node starts them (-):
//   Q(d, 0): +-t (e^{i d jx} + e^{i d jy}),   Q(0, w) i w: +-2 e^{i w t};
// the top boundary node of subspin x ends a segment at beta (+beta e^{i d j};
// at w = 2 pi / beta its e^{i w beta} = 1 cancels the bottom node's 1).
// The bottom (tau = 0+) nodes give the equal-time P_c = sum e^{i d j}.
//
// Pass: (1) flag the loops' smallest nodes and scan them into loop indices; (2) every node adds its terms to its loop's
// record (FP64 atomics); (3) squares summed per loop.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lc_kernels.h"

namespace {

constexpr int kFB = 256;
constexpr int kRec = 7;  // Q(0,0); Q(d,0) re, im; i w Q(0,w) re, im; P re, im

struct FourierCtx {
  const int64_t* parent;
  const int64_t* loopidx;
  int64_t node_base;
};

// Loop index of chain-local node v: its label (the loop's smallest node,
// through at most two parent words) numbered by the scan of the roots.
__device__ inline int64_t loop_of(const FourierCtx& F, int64_t v) {
  const int64_t g = F.node_base + v;
  const int64_t p = F.parent[g];
  int64_t lab = g;
  if (lc::is_closed_word(p)) {
    lab = lc::closed_rep(p);
  } else if (p >= 0) {
    const int64_t pp = F.parent[p];
    lab = pp >= 0 ? pp : p;
  }
  return F.loopidx[lab - F.node_base];
}

// a loop's smallest node: a loop code, or a finished loop's code naming it
__global__ __launch_bounds__(kFB) void k_four_flag(LcFourierArgs A) {
  for (int64_t v = static_cast<int64_t>(blockIdx.x) * kFB + threadIdx.x; v <= A.n_nodes;
       v += static_cast<int64_t>(gridDim.x) * kFB) {
    int64_t f = 0;
    if (v < A.n_nodes) {
      const int64_t g = A.node_base + v, p = A.parent[g];
      f = p < 0 && (!lc::is_closed_word(p) || lc::closed_rep(p) == g) ? 1 : 0;
    }
    A.loopidx[v] = f;
  }
}

__global__ __launch_bounds__(kFB) void k_four_ops(LcFourierArgs A) {
  const FourierCtx F{A.parent, A.loopidx, A.node_base};
  const int64_t ts = A.two_s, W = int64_t(1) << A.w, nw = A.n_bonds * W;
  const double d = 2.0 / static_cast<double>(A.L);  // site phase d j = pi (2 j / L)
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kFB + threadIdx.x; i < nw;
       i += static_cast<int64_t>(gridDim.x) * kFB) {
    const int64_t b = i >> A.w;
    const int64_t j = b / ts / ts;  // bond (j ts + a) ts + c joins sites j and j + 1
    const int64_t jy = j + 1 == A.L ? 0 : j + 1;
    double sx, cx, sy, cy;
    sincospi(d * static_cast<double>(j), &sx, &cx);
    sincospi(d * static_cast<double>(jy), &sy, &cy);
    for (int64_t q = A.opstart[A.win_base + i]; q < A.opstart[A.win_base + i + 1]; ++q) {
      const uint64_t t = A.optime[q];
      const double f = ldexp(static_cast<double>(t), -64);  // t / 2^64
      const double tb = f * A.beta;
      double sw, cw;
      sincospi(2.0 * f, &sw, &cw);
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const double sg = h ? -1.0 : 1.0;  // lower node ends its segments, upper starts them
        const int64_t li = loop_of(F, A.nbn + 2 * (q - A.op_base) + h);
        double* r = A.acc + kRec * li;
        atomicAdd(r + 0, sg * 2.0 * tb);
        atomicAdd(r + 1, sg * tb * (cx + cy));
        atomicAdd(r + 2, sg * tb * (sx + sy));
        atomicAdd(r + 3, sg * 2.0 * cw);
        atomicAdd(r + 4, sg * 2.0 * sw);
      }
    }
  }
}

__global__ __launch_bounds__(kFB) void k_four_bnodes(LcFourierArgs A) {
  const FourierCtx F{A.parent, A.loopidx, A.node_base};
  const double d = 2.0 / static_cast<double>(A.L);
  for (int64_t x = static_cast<int64_t>(blockIdx.x) * kFB + threadIdx.x; x < A.n_sites;
       x += static_cast<int64_t>(gridDim.x) * kFB) {
    const int64_t j = x / A.two_s;
    double s, c;
    sincospi(d * static_cast<double>(j), &s, &c);
    double* rb = A.acc + kRec * loop_of(F, x);  // bottom node: tau = 0+
    atomicAdd(rb + 5, c);
    atomicAdd(rb + 6, s);
    double* rt = A.acc + kRec * loop_of(F, A.two_s == 1 ? x : A.n_sites + x);  // top node: beta
    atomicAdd(rt + 0, A.beta);
    atomicAdd(rt + 1, A.beta * c);
    atomicAdd(rt + 2, A.beta * s);
  }
}

__device__ inline double block_sum_f64(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kFB / 64; ++w) t += sh[w];
  __syncthreads();
  return t;  // valid in thread 0
}

__global__ __launch_bounds__(kFB) void k_four_sums(LcFourierArgs A, int64_t n_loops) {
  __shared__ double sh[kFB / 64];
  double s[4] = {0, 0, 0, 0};
  for (int64_t l = static_cast<int64_t>(blockIdx.x) * kFB + threadIdx.x; l < n_loops;
       l += static_cast<int64_t>(gridDim.x) * kFB) {
    const double* r = A.acc + kRec * l;
    s[0] += r[0] * r[0];
    s[1] += r[1] * r[1] + r[2] * r[2];
    s[2] += r[3] * r[3] + r[4] * r[4];
    s[3] += r[5] * r[5] + r[6] * r[6];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double t = block_sum_f64(s[k], sh);
    if (threadIdx.x == 0) atomicAdd(A.out + k, t);
  }
}

__global__ void k_four_zero(double* p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0;
}

int grid_for(int64_t n) {
  const int64_t b = (n + kFB - 1) / kFB;
  return static_cast<int>(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

hipError_t lc_launch_fourier_index(const LcFourierArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_four_flag, dim3(grid_for(A.n_nodes + 1)), dim3(kFB), 0, s, A);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return lc_launch_scan(A.loopidx, A.n_nodes, A.scan_tmp, s);
}

hipError_t lc_launch_fourier_sums(const LcFourierArgs& A, int64_t n_loops, hipStream_t s) {
  hipLaunchKernelGGL(k_four_zero, dim3(grid_for(kRec * n_loops)), dim3(kFB), 0, s, A.acc,
                     static_cast<int64_t>(kRec) * n_loops);
  hipLaunchKernelGGL(k_four_zero, dim3(1), dim3(64), 0, s, A.out, int64_t(4));
  hipLaunchKernelGGL(k_four_ops, dim3(grid_for(A.n_bonds << A.w)), dim3(kFB), 0, s, A);
  hipLaunchKernelGGL(k_four_bnodes, dim3(grid_for(A.n_sites)), dim3(kFB), 0, s, A);
  hipLaunchKernelGGL(k_four_sums, dim3(grid_for(n_loops) < 1024 ? grid_for(n_loops) : 1024), dim3(kFB), 0,
                     s, A, n_loops);
  return hipGetLastError();
}
