// Kernels of the paper's two applications of a stable integer sort
// (Section 6.2): graph transpose (edges sorted stably by target) and Morton
// order (points sorted by z-value).  The sort itself is the library's.
#include <algorithm>

#include "launch.hpp"

namespace dts {

// Validity of a CSR offsets array: offsets[0] = 0, non-decreasing,
// offsets[V] = E.  Sets *err on a violation.
__global__ __launch_bounds__(256) void k_check_csr(const uint64_t* off, uint32_t n_vertices, uint64_t n_edges,
                                                   uint32_t* err) {
  for (uint64_t v = blockIdx.x * 256ull + threadIdx.x; v <= n_vertices; v += (uint64_t)gridDim.x * 256ull) {
    const uint64_t o = off[v];
    bool bad = o > n_edges;
    if (v == 0) bad |= o != 0;
    if (v == n_vertices) bad |= o != n_edges;
    if (v > 0) bad |= off[v - 1] > o;
    if (bad) atomicOr(err, 1u);
  }
}

// Edge e of the CSR graph: key = its target (copied), value = its source u
// (offsets[u] <= e < offsets[u+1]).  Each workgroup takes EPW consecutive
// edges: their sources lie between the vertices of its first and last edge,
// found once; every edge then binary-searches that range.  A target outside
// [0, V) sets *err.
constexpr uint32_t EPW = 4096;
__global__ __launch_bounds__(256) void k_edge_sources(const uint64_t* off, const uint32_t* tgt, uint32_t n_vertices,
                                                      uint64_t n_edges, uint32_t* keys, uint32_t* src, uint32_t* err) {
  __shared__ uint32_t range[2];
  const uint64_t n_blocks = (n_edges + EPW - 1) / EPW;
  // the last vertex u with offsets[u] <= e (among vertices with out-edges)
  auto vertex_of = [&](uint64_t e, uint32_t lo, uint32_t hi) {  // search in [lo, hi]
    uint32_t n = hi - lo + 1;
    while (n > 0) {
      const uint32_t half = n >> 1;
      if (off[lo + half] <= e) {
        lo += half + 1;
        n -= half + 1;
      } else {
        n = half;
      }
    }
    return lo - 1;
  };
  for (uint64_t b = blockIdx.x; b < n_blocks; b += gridDim.x) {
    const uint64_t e0 = b * EPW;
    const uint64_t e1 = min(n_edges, e0 + EPW) - 1;
    if (threadIdx.x == 0) range[0] = vertex_of(e0, 0, n_vertices);
    if (threadIdx.x == 64) range[1] = vertex_of(e1, 0, n_vertices);
    __syncthreads();
    const uint32_t u0 = range[0], u1 = range[1];
    for (uint64_t e = e0 + threadIdx.x; e <= e1; e += 256) {
      const uint32_t t = tgt[e];
      if (t >= n_vertices) atomicOr(err, 2u);
      keys[e] = t;
      src[e] = vertex_of(e, u0, u1 + 1 <= n_vertices ? u1 + 1 : n_vertices);
    }
    __syncthreads();
  }
}

// Offsets of the transposed graph from the edges sorted by target:
// t_off[v] = number of edges with target < v (a lower bound in the sorted keys).
__global__ __launch_bounds__(256) void k_offsets_of_sorted(const uint32_t* keys, uint64_t n_edges, uint32_t n_vertices,
                                                           uint64_t* t_off) {
  for (uint64_t v = blockIdx.x * 256ull + threadIdx.x; v <= n_vertices; v += (uint64_t)gridDim.x * 256ull) {
    uint64_t lo = 0, n = n_edges;
    while (n > 0) {
      const uint64_t half = n >> 1;
      if ((uint64_t)keys[lo + half] < v) {
        lo += half + 1;
        n -= half + 1;
      } else {
        n = half;
      }
    }
    t_off[v] = lo;
  }
}

// Bits 0..15 of x spread to the even bits (bit i -> bit 2i).
__device__ inline uint32_t spread2(uint32_t x) {
  x &= 0x0000FFFFu;
  x = (x | (x << 8)) & 0x00FF00FFu;
  x = (x | (x << 4)) & 0x0F0F0F0Fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

// Bits 0..9 of x spread to every third bit (bit i -> bit 3i).
__device__ inline uint32_t spread3(uint32_t x) {
  x &= 0x000003FFu;
  x = (x | (x << 16)) & 0x030000FFu;
  x = (x | (x << 8)) & 0x0300F00Fu;
  x = (x | (x << 4)) & 0x030C30C3u;
  x = (x | (x << 2)) & 0x09249249u;
  return x;
}

// z-value of point i (coordinate j at coords[j * n + i]) and its index.
__global__ __launch_bounds__(256) void k_morton(const uint32_t* coords, int dims, uint64_t n, uint32_t* codes,
                                                uint32_t* idx) {
  for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < n; i += (uint64_t)gridDim.x * 256ull) {
    uint32_t z;
    if (dims == 2)
      z = spread2(coords[i]) | (spread2(coords[n + i]) << 1);
    else
      z = spread3(coords[i]) | (spread3(coords[n + i]) << 1) | (spread3(coords[2 * n + i]) << 2);
    codes[i] = z;
    idx[i] = (uint32_t)i;
  }
}

static uint32_t grid_for(uint64_t items, uint32_t per_block) {
  const uint64_t g = (items + per_block - 1) / per_block;
  return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(g, persistent_grid(16)));
}

void launch_transpose_prepare(const uint64_t* off, const uint32_t* tgt, uint32_t n_vertices, uint64_t n_edges,
                              uint32_t* keys, uint32_t* src, uint32_t* err, hipStream_t s) {
  hipLaunchKernelGGL(k_check_csr, dim3(grid_for((uint64_t)n_vertices + 1, 256)), dim3(256), 0, s, off, n_vertices,
                     n_edges, err);
  if (n_edges == 0) return;
  hipLaunchKernelGGL(k_edge_sources, dim3(grid_for(n_edges, EPW)), dim3(256), 0, s, off, tgt, n_vertices, n_edges,
                     keys, src, err);
}

void launch_transpose_offsets(const uint32_t* keys, uint64_t n_edges, uint32_t n_vertices, uint64_t* t_off,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_offsets_of_sorted, dim3(grid_for((uint64_t)n_vertices + 1, 256)), dim3(256), 0, s, keys,
                     n_edges, n_vertices, t_off);
}

void launch_morton(const uint32_t* coords, int dims, uint64_t n, uint32_t* codes, uint32_t* idx, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_morton, dim3(grid_for(n, 256)), dim3(256), 0, s, coords, dims, n, codes, idx);
}

}  // namespace dts
