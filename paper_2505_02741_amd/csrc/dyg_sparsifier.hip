// Initial sparsifier H(0) on the GPU: the input of the update path (Algorithm
// 1 starts from a sparsifier H(0) of G(0); the experiments build it with
// GRASS, Sec. IV-A, whose spanning-tree-plus-off-tree-edges structure this
// follows).
//
//   1. Maximum spanning forest by Boruvka rounds: every component takes its
//      heaviest incident edge, ties to the smaller canonical edge index (a
//      strict order, so every edge taken is in the unique forest Kruskal
//      would keep under the same order), components hook along them
//      (a pair that took the same edge keeps the smaller id as root), and
//      pointer jumping relabels every vertex; until no component has an
//      edge leaving it.
//   2. Off-tree sample: every edge outside the forest draws a 64-bit key from
//      Philox-4x32-10 (key = seed, counter = (edge index, 0, a tag word));
//      the n_extra smallest keys, ties to the smaller index, are taken: a
//      uniform sample without replacement.  A histogram of the top 16 key
//      bits finds the bucket where the n_extra-th key lies; the buckets
//      below it are taken whole on the device, and that one bucket's
//      candidates (a few thousand at most for random keys) are ordered on
//      the host.
//
// Canonical edges: the pairs (u, v), u < v, of the CSR in ascending (u, v)
// order; edge e is the e-th.
#include "dygrass.h"
#include "dyg_internal.h"
#include "dyg_philox.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

namespace dyg {
namespace {

constexpr int kSpBlock = 256;
constexpr uint32_t kSampleTag = 0x53504152u;  // counter word 3 of the sample keys
constexpr uint32_t kBucketBits = 16;
constexpr uint32_t kNoEdge = 0xFFFFFFFFu;

__device__ __forceinline__ unsigned long long weight_bits(double w) {
  // w > 0: the IEEE bit pattern orders like the value
  return static_cast<unsigned long long>(__double_as_longlong(w));
}

__device__ __forceinline__ unsigned long long sample_key(uint64_t seed, uint64_t e) {
  const Philox4 x = philox4x32_10(static_cast<uint32_t>(e), static_cast<uint32_t>(e >> 32), 0u,
                                  kSampleTag, static_cast<uint32_t>(seed),
                                  static_cast<uint32_t>(seed >> 32));
  return static_cast<unsigned long long>(x.x0) | (static_cast<unsigned long long>(x.x1) << 32);
}

__global__ void k_sp_init(uint32_t n, uint32_t* comp) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) comp[v] = v;
}

// Start of a round: no component has a candidate edge yet.
__global__ void k_sp_clear(uint32_t n, unsigned long long* bestw, uint32_t* beste,
                           unsigned int* hooks) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c == 0) *hooks = 0;
  if (c < n) {
    bestw[c] = 0ull;
    beste[c] = kNoEdge;
  }
}

// Heaviest weight leaving each component.
__global__ void k_sp_best_w(uint64_t m, const uint32_t* __restrict__ eu,
                            const uint32_t* __restrict__ ev, const double* __restrict__ ew,
                            const uint32_t* __restrict__ comp, unsigned long long* bestw) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= m) return;
  const uint32_t a = comp[eu[e]], b = comp[ev[e]];
  if (a == b) return;
  const unsigned long long wb = weight_bits(ew[e]);
  if (wb > bestw[a]) atomicMax(&bestw[a], wb);
  if (wb > bestw[b]) atomicMax(&bestw[b], wb);
}

// Among the edges of that weight, the smallest index.
__global__ void k_sp_best_e(uint64_t m, const uint32_t* __restrict__ eu,
                            const uint32_t* __restrict__ ev, const double* __restrict__ ew,
                            const uint32_t* __restrict__ comp,
                            const unsigned long long* __restrict__ bestw, uint32_t* beste) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= m) return;
  const uint32_t a = comp[eu[e]], b = comp[ev[e]];
  if (a == b) return;
  const unsigned long long wb = weight_bits(ew[e]);
  if (wb == bestw[a]) atomicMin(&beste[a], static_cast<uint32_t>(e));
  if (wb == bestw[b]) atomicMin(&beste[b], static_cast<uint32_t>(e));
}

// Each root with a candidate hooks onto the root at the edge's other end and
// puts the edge in the forest; when two roots took the same edge, the
// smaller id stays root.  nxt holds the new parent of every root.
__global__ void k_sp_hook(uint32_t n, const uint32_t* __restrict__ eu,
                          const uint32_t* __restrict__ ev, const uint32_t* __restrict__ comp,
                          const uint32_t* __restrict__ beste, uint32_t* nxt, uint8_t* in_f,
                          unsigned int* hooks) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || comp[c] != c) return;  // roots only
  const uint32_t e = beste[c];
  if (e == kNoEdge) {
    nxt[c] = c;
    return;
  }
  const uint32_t a = comp[eu[e]], b = comp[ev[e]];
  const uint32_t other = a == c ? b : a;
  in_f[e] = 1;
  const bool mutual = beste[other] == e;
  nxt[c] = (mutual && c < other) ? c : other;
  atomicAdd(hooks, 1u);
}

// Pointer jumping over the roots' parents: nxt[c] = nxt[nxt[c]] until every
// root points at a root of the merged component.
__global__ void k_sp_jump(uint32_t n, const uint32_t* __restrict__ comp, uint32_t* nxt,
                          unsigned int* changed) {
  const uint32_t c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || comp[c] != c) return;
  const uint32_t p = nxt[c], g = nxt[p];
  if (g != p) {
    nxt[c] = g;
    *changed = 1u;
  }
}

__global__ void k_sp_relabel(uint32_t n, uint32_t* comp, const uint32_t* __restrict__ nxt) {
  const uint32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) comp[v] = nxt[comp[v]];
}

// Histogram of the top key bits of the edges outside the forest.
__global__ void k_sp_hist(uint64_t m, const uint8_t* __restrict__ in_f, uint64_t seed,
                          unsigned int* hist) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= m || in_f[e]) return;
  atomicAdd(&hist[sample_key(seed, e) >> (64 - kBucketBits)], 1u);
}

struct Cand {
  unsigned long long key;
  uint64_t e;
};

// Buckets below `bucket` are taken whole (flag 2); that bucket's edges are
// listed for the host to order.
__global__ void k_sp_select(uint64_t m, uint8_t* in_f, uint64_t seed, uint32_t bucket,
                            Cand* cand, unsigned int* ncand) {
  const uint64_t e = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x;
  if (e >= m || in_f[e]) return;
  const unsigned long long key = sample_key(seed, e);
  const uint32_t b = static_cast<uint32_t>(key >> (64 - kBucketBits));
  if (b < bucket) in_f[e] = 2;
  else if (b == bucket) cand[atomicAdd(ncand, 1u)] = Cand{key, e};
}

inline uint32_t grid(uint64_t x) { return static_cast<uint32_t>((x + kSpBlock - 1) / kSpBlock); }

struct DevMem {
  std::vector<void*> p;
  ~DevMem() {
    for (void* q : p) (void)hipFree(q);
  }
  template <class T>
  T* get(size_t count, hipError_t& e) {
    void* q = nullptr;
    if (e == hipSuccess) e = hipMalloc(&q, sizeof(T) * std::max<size_t>(count, 1));
    if (e == hipSuccess) p.push_back(q);
    return static_cast<T*>(q);
  }
};

int fail(hipError_t e) { return e == hipErrorOutOfMemory ? DYG_E_NOMEM : DYG_E_DEVICE; }

// Flags per canonical edge: 1 = forest, 2 = sampled, 0 = neither.
int build_flags(uint32_t n, const std::vector<uint32_t>& eu, const std::vector<uint32_t>& ev,
                const std::vector<double>& ew, uint64_t n_extra, uint64_t seed,
                std::vector<uint8_t>& flags) {
  const uint64_t m = eu.size();
  flags.assign(m, 0);
  if (m == 0) return DYG_OK;
  hipStream_t st = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return fail(e);
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() { (void)hipStreamDestroy(s); }
  } guard{st};
  DevMem mem;
  uint32_t* d_eu = mem.get<uint32_t>(m, e);
  uint32_t* d_ev = mem.get<uint32_t>(m, e);
  double* d_ew = mem.get<double>(m, e);
  uint8_t* d_in = mem.get<uint8_t>(m, e);
  uint32_t* comp = mem.get<uint32_t>(n, e);
  uint32_t* nxt = mem.get<uint32_t>(n, e);
  unsigned long long* bestw = mem.get<unsigned long long>(n, e);
  uint32_t* beste = mem.get<uint32_t>(n, e);
  unsigned int* ctr = mem.get<unsigned int>(4, e);  // hooks, changed, candidates
  unsigned int* hist = mem.get<unsigned int>(size_t(1) << kBucketBits, e);
  if (e != hipSuccess) return fail(e);
  if ((e = hipMemcpyAsync(d_eu, eu.data(), 4 * m, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(d_ev, ev.data(), 4 * m, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(d_ew, ew.data(), 8 * m, hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemsetAsync(d_in, 0, m, st)) != hipSuccess)
    return fail(e);
  k_sp_init<<<grid(n), kSpBlock, 0, st>>>(n, comp);
  // Boruvka rounds: each at least halves the components that still have an
  // edge leaving them, so at most log2(n) + 1 rounds do any work
  for (int round = 0; round < 64; ++round) {
    k_sp_clear<<<grid(n), kSpBlock, 0, st>>>(n, bestw, beste, ctr);
    k_sp_best_w<<<grid(m), kSpBlock, 0, st>>>(m, d_eu, d_ev, d_ew, comp, bestw);
    k_sp_best_e<<<grid(m), kSpBlock, 0, st>>>(m, d_eu, d_ev, d_ew, comp, bestw, beste);
    k_sp_hook<<<grid(n), kSpBlock, 0, st>>>(n, d_eu, d_ev, comp, beste, nxt, d_in, ctr);
    unsigned int hooks = 0;
    if ((e = hipMemcpyAsync(&hooks, ctr, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return fail(e);
    if (hooks == 0) break;
    // every hook chain ends at a root that kept itself: at most n jumps of
    // doubling length, far fewer in practice
    for (uint32_t j = 0; j < 64; ++j) {
      unsigned int changed = 0;
      if ((e = hipMemsetAsync(ctr + 1, 0, 4, st)) != hipSuccess) return fail(e);
      k_sp_jump<<<grid(n), kSpBlock, 0, st>>>(n, comp, nxt, ctr + 1);
      if ((e = hipMemcpyAsync(&changed, ctr + 1, 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
          (e = hipStreamSynchronize(st)) != hipSuccess)
        return fail(e);
      if (!changed) break;
    }
    k_sp_relabel<<<grid(n), kSpBlock, 0, st>>>(n, comp, nxt);
  }
  if ((e = hipGetLastError()) != hipSuccess) return fail(e);
  std::vector<Cand> cands;
  if (n_extra > 0) {
    if ((e = hipMemsetAsync(hist, 0, sizeof(unsigned int) << kBucketBits, st)) != hipSuccess)
      return fail(e);
    k_sp_hist<<<grid(m), kSpBlock, 0, st>>>(m, d_in, seed, hist);
    std::vector<unsigned int> h(size_t(1) << kBucketBits);
    if ((e = hipMemcpyAsync(h.data(), hist, sizeof(unsigned int) * h.size(),
                            hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return fail(e);
    // the bucket holding the n_extra-th smallest key (or one past the last)
    uint64_t below = 0;
    uint32_t bucket = 0;
    while (bucket < h.size() && below + h[bucket] < n_extra) below += h[bucket++];
    const uint32_t in_bucket = bucket < h.size() ? h[bucket] : 0u;
    Cand* cand = mem.get<Cand>(in_bucket, e);
    if (e != hipSuccess) return fail(e);
    if ((e = hipMemsetAsync(ctr + 2, 0, 4, st)) != hipSuccess) return fail(e);
    k_sp_select<<<grid(m), kSpBlock, 0, st>>>(m, d_in, seed, bucket, cand, ctr + 2);
    if ((e = hipGetLastError()) != hipSuccess) return fail(e);
    cands.resize(in_bucket);
    if (in_bucket &&
        (e = hipMemcpyAsync(cands.data(), cand, sizeof(Cand) * in_bucket, hipMemcpyDeviceToHost,
                            st)) != hipSuccess)
      return fail(e);
    std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) {
      return x.key != y.key ? x.key < y.key : x.e < y.e;
    });
    cands.resize(std::min<uint64_t>(cands.size(), n_extra - below));
  }
  if ((e = hipMemcpyAsync(flags.data(), d_in, m, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return fail(e);
  for (const Cand& c : cands) flags[c.e] = 2;
  return DYG_OK;
}

}  // namespace
}  // namespace dyg

extern "C" int dyg_initial_sparsifier(uint32_t n, const uint64_t* rowptr, const uint32_t* col,
                                      const double* w, uint64_t n_extra, uint64_t seed,
                                      uint64_t cap, uint64_t* m_out, uint32_t* h_u,
                                      uint32_t* h_v) {
  if (!m_out || (cap && (!h_u || !h_v))) return DYG_E_INVALID_ARG;
  int rc = dyg::validate_csr(n, rowptr, col, w, nullptr);
  if (rc) return rc;
  if (rowptr[n] / 2 >= (1ull << 32)) return DYG_E_INVALID_ARG;  // edge ids are 32-bit
  std::vector<uint32_t> eu, ev;
  std::vector<double> ew;
  eu.reserve(rowptr[n] / 2);
  ev.reserve(rowptr[n] / 2);
  ew.reserve(rowptr[n] / 2);
  for (uint32_t u = 0; u < n; ++u)
    for (uint64_t k = rowptr[u]; k < rowptr[u + 1]; ++k)
      if (col[k] > u) {
        eu.push_back(u);
        ev.push_back(col[k]);
        ew.push_back(w[k]);
      }
  std::vector<uint8_t> flags;
  rc = dyg::build_flags(n, eu, ev, ew, n_extra, seed, flags);
  if (rc) return rc;
  uint64_t count = 0;
  for (uint8_t f : flags) count += f != 0;
  *m_out = count;
  if (cap < count) return DYG_OK;
  uint64_t o = 0;
  for (uint64_t e = 0; e < flags.size(); ++e)
    if (flags[e]) {
      h_u[o] = eu[e];
      h_v[o] = ev[e];
      ++o;
    }
  return DYG_OK;
}
