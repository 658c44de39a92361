// dcs_graph.hip -- random graphs G(n, m) and G(n, p) (Sec. 7: generating
// such a graph is sampling from its n(n-1)/2 possible edges, without
// replacement for G(n, m) and by Bernoulli sampling for G(n, p)).
//
// The edge with index k (0-based) is the pair (u, v), v < u, with
// k = u(u-1)/2 + v: edges ordered by u, then v.  The sampler writes sorted
// 1-based indices; one elementwise kernel turns each 8-byte index in place
// into the two 32-bit vertex numbers (u, v), so the edge list keeps the
// sample's order and needs no buffer beyond the caller's.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <mutex>

#include "../../include/dcs.h"
#include "dcs_host.hpp"

namespace dcs {

// Pair (u, v) of edge index k < 2^62: u is the integer with
// u(u-1)/2 <= k < u(u+1)/2, i.e. the floor of (1 + sqrt(8k+1))/2.  The FP64
// root of 8k+1 (formed in double, below 2^65; relative error near 2^-52)
// puts the floor within one of u (u < 2^32), and at most one step of
// integer comparison against the triangular numbers (products below 2^64)
// each way makes it exact; two are allowed.  An index outside that range
// (no sample value produces one) gives the pair (2^32-1, 2^32-1) instead of
// an unbounded correction.
__device__ __forceinline__ uint64_t edge_pair(uint64_t k) {
  if (k >= (1ull << 62)) return ~0ull;
  const double r = sqrt(8.0 * static_cast<double>(k) + 1.0);
  uint64_t u = static_cast<uint64_t>((1.0 + r) * 0.5);
#pragma unroll
  for (int i = 0; i < 2; ++i)
    if (u > 1 && u * (u - 1) / 2 > k) --u;
#pragma unroll
  for (int i = 0; i < 2; ++i)
    if (u * (u + 1) / 2 <= k) ++u;
  const uint64_t v = k - u * (u - 1) / 2;
  return u | (v << 32);  // little endian: u at the lower address
}

// In place over x[0..min(n, *count)) (count == null: all n): sample value
// k+1 -> packed (u, v).  Grid-stride; consecutive lanes on consecutive words.
__global__ __launch_bounds__(256) void k_edge_decode(uint64_t* x, uint64_t n,
                                                     const uint64_t* count) {
  uint64_t total = n;
  if (count != nullptr) total = std::min<uint64_t>(n, *count);
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < total;
       i += stride) {
    const uint64_t k = __builtin_nontemporal_load(x + i) - 1;
    __builtin_nontemporal_store(edge_pair(k), x + i);
  }
}

}  // namespace dcs

namespace {

using namespace dcs::host;

// Edges of a graph on n vertices, or an error if n(n-1)/2 exceeds the
// largest universe of the sampler used (max_N).
int32_t edge_universe(uint64_t n_vertices, uint64_t max_N, uint64_t* N) {
  if (n_vertices > (1ull << 32)) return DCS_EINVAL;
  const uint64_t e = n_vertices < 2 ? 0 : n_vertices * (n_vertices - 1) / 2;
  if (e > max_N) return DCS_EINVAL;
  *N = e;
  return DCS_OK;
}

int32_t launch_decode(uint64_t* x, uint64_t n, const uint64_t* count, hipStream_t s) {
  if (n == 0) return DCS_OK;
  std::lock_guard<std::mutex> lk(lock());
  DeviceCtx* c;
  int32_t rc = device_ctx(&c);
  if (rc) return rc;
  const uint64_t want = (n + 255) / 256;
  const uint64_t cap = static_cast<uint64_t>(c->cus) * 16;  // enough waves to fill HBM
  const uint32_t blocks = static_cast<uint32_t>(std::max<uint64_t>(1, std::min(want, cap)));
  Timing t{};
  timing_begin(7, s, &t);
  hipLaunchKernelGGL(dcs::k_edge_decode, dim3(blocks), dim3(256), 0, s, x, n, count);
  const hipError_t e = hipGetLastError();
  timing_end(s, &t);
  return e == hipSuccess ? DCS_OK : DCS_EHIP;
}

}  // namespace

extern "C" {

int32_t dcs_sample_edges_gnm(uint64_t n_vertices, uint64_t m, uint64_t seed,
                             const dcs_params* params, uint32_t* uv_dev, void* stream) {
  uint64_t N = 0;
  if (edge_universe(n_vertices, DCS_MAX_UNIVERSE, &N) != DCS_OK || m > N) return DCS_EINVAL;
  if (m > 0 && (uv_dev == nullptr || (reinterpret_cast<uintptr_t>(uv_dev) & 7u) != 0))
    return DCS_EINVAL;
  if (m == 0) return DCS_OK;
  uint64_t* x = reinterpret_cast<uint64_t*>(uv_dev);
  int32_t rc = dcs_sample_ex(m, N, seed, params, x, nullptr, 0, stream);
  if (rc) return rc;
  return launch_decode(x, m, nullptr, static_cast<hipStream_t>(stream));
}

int32_t dcs_sample_edges_gnp(uint64_t n_vertices, double p, uint64_t seed,
                             const dcs_params* params, uint32_t* uv_dev, uint64_t capacity,
                             uint64_t* count_dev, void* stream) {
  uint64_t N = 0;
  if (edge_universe(n_vertices, DCS_MAX_BERNOULLI_UNIVERSE, &N) != DCS_OK) return DCS_EINVAL;
  if (capacity > 0 && (uv_dev == nullptr || (reinterpret_cast<uintptr_t>(uv_dev) & 7u) != 0))
    return DCS_EINVAL;
  uint64_t* x = reinterpret_cast<uint64_t*>(uv_dev);
  int32_t rc = dcs_sample_bernoulli_ex(p, N, seed, params, x, capacity, count_dev, nullptr, 0,
                                       stream);
  if (rc) return rc;
  return launch_decode(x, capacity, count_dev, static_cast<hipStream_t>(stream));
}

}  // extern "C"
