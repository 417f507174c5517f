// Bound storage (Sec. 6.1): group the leaves by tuple and splat every leaf's
// irradiance bound into the receiver-grid cells its closed position bound
// touches, keeping per (cell, tuple) the maximum (Eq. eq_pertuple_b, m = 1).
// The grid is a CSR: offsets per cell, then (tuple, E~) sorted by tuple.
//
// Kernels (all counts read from device memory, no host synchronisation):
//   k_leaf_count / scan / k_leaf_scatter / k_leaf_rank   leaves grouped by tuple
//   k_grid_tuple   one 256-thread workgroup per tuple: the union of its leaves'
//                  cell rectangles is rasterised in LDS bands with an atomic
//                  max, then the occupied cells are emitted as triples
//   scan / k_grid_scatter / k_grid_rank                   triples -> CSR by cell
//   k_tuple_records  one packed 128-byte record per tuple for the query stage
#include "internal.hpp"

namespace bbc {

// ---------------------------------------------------------------- exclusive scan
constexpr int kScanThreads = 256, kScanItems = 8, kScanTile = kScanThreads * kScanItems;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* total) {
  __shared__ uint32_t wsum[kScanThreads / BBC_WAVE];
  const int lane = threadIdx.x % BBC_WAVE, w = threadIdx.x / BBC_WAVE;
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < BBC_WAVE; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d, BBC_WAVE);
    if (lane >= d) inc += o;
  }
  if (lane == BBC_WAVE - 1) wsum[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int i = 0; i < kScanThreads / BBC_WAVE; ++i) {
    if (i < w) off += wsum[i];
    tot += wsum[i];
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_sums(const uint32_t* in, int64_t n, uint32_t* sums) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile;
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + int64_t(k) * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
  uint32_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

// Exclusive scan of the block sums in one workgroup (up to 256 * 64 blocks).
__global__ void __launch_bounds__(kScanThreads) k_scan_top(uint32_t* sums, int64_t nb) {
  const int64_t per = (nb + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = threadIdx.x * per;
  uint32_t s = 0;
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) s += sums[b0 + i];
  uint32_t tot;
  uint32_t off = block_exclusive_scan(s, &tot);
  for (int64_t i = 0; i < per; ++i)
    if (b0 + i < nb) {
      const uint32_t v = sums[b0 + i];
      sums[b0 + i] = off;
      off += v;
    }
  if (threadIdx.x == 0) sums[nb] = tot;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const uint32_t* in, int64_t n, const uint32_t* sums,
                                                             uint32_t* out, int64_t nb) {
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint32_t s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    v[k] = i < n ? in[i] : 0u;
    s += v[k];
  }
  uint32_t tot;
  uint32_t off = block_exclusive_scan(s, &tot) + sums[blockIdx.x];
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t i = base + k;
    if (i < n) out[i] = off;
    off += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

size_t scan_tmp_bytes(int64_t n) { return size_t((n + kScanTile - 1) / kScanTile + 1) * 4; }

bbc_status launch_scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp, hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanTile - 1) / kScanTile);
  if (nb > int64_t(kScanThreads) * 4096) return BBC_EINVAL;
  uint32_t* sums = static_cast<uint32_t*>(tmp);
  hipLaunchKernelGGL(k_scan_sums, dim3(unsigned(nb)), dim3(kScanThreads), 0, s, in, n, sums);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, sums, nb);
  hipLaunchKernelGGL(k_scan_apply, dim3(unsigned(nb)), dim3(kScanThreads), 0, s, in, n, sums, out, nb);
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

// ---------------------------------------------------------------- leaves by tuple
struct RecArgs {
  BuildCounters* C;
  int64_t n_tuples;
  uint32_t leaf_cap, trip_cap;
  int G;
  const uint32_t* lt;
  const uint32_t* lc;
  const float4* lu;
  const float2* le;
  uint32_t* tcount;
  uint32_t* toff;
  uint32_t* tcur;
  uint32_t* gt_;  // leaves grouped by tuple (arbitrary order inside a tuple)
  uint32_t* gc;
  float4* gu;
  float2* ge_;
  uint32_t* st;   // leaves grouped by tuple, ordered by code
  uint32_t* sc;
  float4* su;
  float2* se;
  uint32_t* trip;  // [3][trip_cap]: cell, tuple, E bits
  uint32_t* ccount;
  uint32_t* coff;
  uint32_t* ccur;
  uint32_t* ut;     // entries grouped by cell, arbitrary order inside a cell
  float* ue;
  uint32_t* ucell;
  uint32_t* gt;     // final entries, sorted by tuple inside each cell
  float* ge;
  uint32_t* max_cell;
};

__global__ void k_leaf_count(RecArgs a) {
  const uint32_t n = min(a.C->n_leaves, a.leaf_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    atomicAdd(&a.tcount[a.lt[i]], 1u);
}

__global__ void k_leaf_scatter(RecArgs a) {
  const uint32_t n = min(a.C->n_leaves, a.leaf_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t t = a.lt[i];
    const uint32_t p = a.toff[t] + atomicAdd(&a.tcur[t], 1u);
    a.gt_[p] = t;
    a.gc[p] = a.lc[i];
    a.gu[p] = a.lu[i];
    a.ge_[p] = a.le[i];
  }
}

// Order each tuple's leaves by their (depth, iu, iv) code, which is unique
// within a tuple: a leaf's final slot is its segment start plus the number of
// smaller codes in the segment.  Every later use is then deterministic.
__global__ void k_leaf_rank(RecArgs a) {
  const uint32_t n = min(a.C->n_leaves, a.leaf_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t t = a.gt_[i], c = a.gc[i];
    const uint32_t b = a.toff[t], e = a.toff[t + 1];
    uint32_t r = 0;
    for (uint32_t j = b; j < e; ++j) r += a.gc[j] < c ? 1u : 0u;
    a.st[b + r] = t;
    a.sc[b + r] = c;
    a.su[b + r] = a.gu[i];
    a.se[b + r] = a.ge_[i];
  }
}

// ---------------------------------------------------------------- receiver grid
__device__ __forceinline__ int cell_of(float x, int G) {
  const float c = floorf(fminf(fmaxf(x, 0.f), 1.f) * float(G));  // NaN maps to 0
  return min(G - 1, max(0, int(c)));
}

constexpr int kGridThreads = 256;
constexpr int kTile = 16384;  // cells rasterised per LDS band

// Triple slots are reserved in chunks of kTripChunk per workgroup (one global
// atomic per chunk, not per tuple); unused slots of a chunk are marked with
// kNoCell and skipped by the scatter.
constexpr uint32_t kTripChunk = 256, kNoCell = 0xffffffffu;

__device__ void mark_unused(const RecArgs& a, uint32_t b, uint32_t e) {
  for (uint32_t i = b + threadIdx.x; i < e && i < a.trip_cap; i += kGridThreads) a.trip[i] = kNoCell;
}

__global__ void __launch_bounds__(kGridThreads) k_grid_tuple(RecArgs a) {
  __shared__ uint32_t tile[kTile];
  __shared__ int rect[4];
  __shared__ uint32_t base_slot, chunk_b, chunk_e, drop_b, drop_e, n_real;
  const int G = a.G;
  if (threadIdx.x == 0) chunk_b = chunk_e = n_real = 0u;
  __syncthreads();
  for (int64_t t = blockIdx.x; t < a.n_tuples; t += gridDim.x) {
    const uint32_t lb = a.toff[t], le = a.toff[t + 1];
    if (lb == le) continue;
    // union of the leaves' cell rectangles
    int cu0 = G, cu1 = -1, cv0 = G, cv1 = -1;
    for (uint32_t k = lb + threadIdx.x; k < le; k += kGridThreads) {
      const float4 u = a.su[k];
      cu0 = min(cu0, cell_of(u.x, G));
      cu1 = max(cu1, cell_of(u.y, G));
      cv0 = min(cv0, cell_of(u.z, G));
      cv1 = max(cv1, cell_of(u.w, G));
    }
    cu0 = wave_min(cu0); cu1 = wave_max(cu1); cv0 = wave_min(cv0); cv1 = wave_max(cv1);
    if (threadIdx.x == 0) { rect[0] = G; rect[1] = -1; rect[2] = G; rect[3] = -1; }
    __syncthreads();
    if (threadIdx.x % BBC_WAVE == 0) {
      atomicMin(&rect[0], cu0); atomicMax(&rect[1], cu1); atomicMin(&rect[2], cv0); atomicMax(&rect[3], cv1);
    }
    __syncthreads();
    cu0 = rect[0]; cu1 = rect[1]; cv0 = rect[2]; cv1 = rect[3];
    const int W = cv1 - cv0 + 1;
    const int rows = max(1, kTile / W);
    __syncthreads();
    for (int r0 = cu0; r0 <= cu1; r0 += rows) {
      const int r1 = min(cu1, r0 + rows - 1);
      const int ncell = (r1 - r0 + 1) * W;
      for (int i = threadIdx.x; i < ncell; i += kGridThreads) tile[i] = 0u;
      __syncthreads();
      for (uint32_t k = lb; k < le; ++k) {
        const float4 u = a.su[k];
        const int a0 = max(r0, cell_of(u.x, G)), a1 = min(r1, cell_of(u.y, G));
        if (a0 > a1) continue;
        const int b0 = cell_of(u.z, G), b1 = cell_of(u.w, G);
        const int bw = b1 - b0 + 1;
        const uint32_t key = __float_as_uint(a.se[k].y) + 1u;  // E_hi >= 0: bit order is value order
        const int cnt = (a1 - a0 + 1) * bw;
        for (int i = threadIdx.x; i < cnt; i += kGridThreads) {
          const int ru = a0 + i / bw, cv = b0 + i % bw;
          atomicMax(&tile[(ru - r0) * W + (cv - cv0)], key);
        }
      }
      __syncthreads();
      // emit the occupied cells of the band
      uint32_t mine = 0;
      for (int i = threadIdx.x; i < ncell; i += kGridThreads) mine += tile[i] != 0u;
      uint32_t tot;
      uint32_t off = block_exclusive_scan(mine, &tot);
      if (threadIdx.x == 0) {
        drop_b = drop_e = 0u;
        if (tot > chunk_e - chunk_b) {  // a fresh chunk; the rest of the old one is marked unused
          drop_b = chunk_b;
          drop_e = chunk_e;
          const uint32_t want = max(tot, kTripChunk);
          chunk_b = atomicAdd(&a.C->n_triples, want);
          chunk_e = chunk_b + want;
        }
        base_slot = chunk_b;
        chunk_b += tot;
        n_real += tot;
      }
      __syncthreads();
      mark_unused(a, drop_b, drop_e);
      const uint32_t bs = base_slot;
      if (bs + tot > a.trip_cap) {
        if (threadIdx.x == 0 && tot) atomicOr(&a.C->overflow, 4u);
      } else {
        for (int i = threadIdx.x; i < ncell; i += kGridThreads) {
          const uint32_t key = tile[i];
          if (!key) continue;
          const uint32_t cell = uint32_t(r0 + i / W) * uint32_t(G) + uint32_t(cv0 + i % W);
          const uint32_t slot = bs + off++;
          a.trip[slot] = cell;
          a.trip[a.trip_cap + slot] = uint32_t(t);
          a.trip[2 * size_t(a.trip_cap) + slot] = key - 1u;
          atomicAdd(&a.ccount[cell], 1u);
        }
      }
      __syncthreads();
    }
  }
  mark_unused(a, chunk_b, chunk_e);
  if (threadIdx.x == 0 && n_real) atomicAdd(&a.C->n_entries, n_real);
}

// Triples -> cells: first grouped by cell in arbitrary order, then each entry
// ranks its tuple id among its cell's entries (tuple ids are unique within a
// cell) and moves to its final slot, so every cell list is sorted by tuple.
__global__ void k_grid_scatter(RecArgs a) {
  const uint32_t n = min(a.C->n_triples, a.trip_cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t cell = a.trip[i];
    if (cell == kNoCell) continue;
    const uint32_t p = a.coff[cell] + atomicAdd(&a.ccur[cell], 1u);
    a.ut[p] = a.trip[a.trip_cap + i];
    a.ue[p] = __uint_as_float(a.trip[2 * size_t(a.trip_cap) + i]);
    a.ucell[p] = cell;
  }
}

__global__ void k_grid_rank(RecArgs a) {
  const uint32_t n = a.coff[uint32_t(a.G) * uint32_t(a.G)];  // entries scattered into the cells
  uint32_t mx = 0;
  for (uint32_t p = blockIdx.x * blockDim.x + threadIdx.x; p < n; p += gridDim.x * blockDim.x) {
    const uint32_t cell = a.ucell[p];
    const uint32_t b = a.coff[cell], e = a.coff[cell + 1];
    const uint32_t t = a.ut[p];
    uint32_t r = 0;
    for (uint32_t j = b; j < e; ++j) r += a.ut[j] < t ? 1u : 0u;
    a.gt[b + r] = t;
    a.ge[b + r] = a.ue[p];
    mx = max(mx, e - b);
  }
  mx = wave_max(mx);
  if (threadIdx.x % BBC_WAVE == 0 && mx) atomicMax(a.max_cell, mx);
}

// One packed record per tuple with leaves (see geom_dev.hpp).
__global__ void k_tuple_records(RecArgs a, DevScene sc, const float4* root, float* rec, int rec_floats) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < a.n_tuples;
       t += int64_t(gridDim.x) * blockDim.x) {
    const uint32_t lb = a.toff[t], le = a.toff[t + 1];
    if (lb == le) continue;
    int64_t first = t;
    float4* r = reinterpret_cast<float4*>(rec + t * rec_floats);
    if (sc.chain == 2) {
      const int64_t dense = sc.tid[t], n2 = sc.n_tri2, t2 = dense % n2;
      first = dense / n2;
      const float* P2 = sc.pos2;
      const float* N2 = sc.nrm2;
      r[7] = make_float4(P2[0 * n2 + t2], P2[1 * n2 + t2], P2[2 * n2 + t2], P2[3 * n2 + t2]);
      r[8] = make_float4(P2[4 * n2 + t2], P2[5 * n2 + t2], P2[6 * n2 + t2], P2[7 * n2 + t2]);
      r[9] = make_float4(P2[8 * n2 + t2], N2[0 * n2 + t2], N2[1 * n2 + t2], N2[2 * n2 + t2]);
      r[10] = make_float4(N2[3 * n2 + t2], N2[4 * n2 + t2], N2[5 * n2 + t2], N2[6 * n2 + t2]);
      r[11] = make_float4(N2[7 * n2 + t2], N2[8 * n2 + t2], 0.f, 0.f);
    } else {
      r[7] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    const int64_t tri = first % sc.n_tri, e = first / sc.n_tri;
    const float* P = sc.pos;
    const float* N = sc.nrm;
    const int64_t n = sc.n_tri;
    r[0] = make_float4(P[0 * n + tri], P[1 * n + tri], P[2 * n + tri], P[3 * n + tri]);
    r[1] = make_float4(P[4 * n + tri], P[5 * n + tri], P[6 * n + tri], P[7 * n + tri]);
    r[2] = make_float4(P[8 * n + tri], N[0 * n + tri], N[1 * n + tri], N[2 * n + tri]);
    r[3] = make_float4(N[3 * n + tri], N[4 * n + tri], N[5 * n + tri], N[6 * n + tri]);
    r[4] = make_float4(N[7 * n + tri], N[8 * n + tri], sc.epos[e], sc.epos[sc.n_emit + e]);
    r[5] = make_float4(sc.epos[2 * sc.n_emit + e], sc.eI[e], __uint_as_float(lb), __uint_as_float(le));
    r[6] = root[t];
  }
}

bbc_status launch_record(Bounds* b, hipStream_t s) {
  RecArgs a{};
  a.C = static_cast<BuildCounters*>(b->counters.p);
  a.n_tuples = b->n_tuples;
  a.leaf_cap = uint32_t(b->leaf_cap);
  a.trip_cap = uint32_t(b->trip_cap);
  a.G = b->params.grid_res;
  a.lt = static_cast<uint32_t*>(b->lt.p);
  a.lc = static_cast<uint32_t*>(b->lc.p);
  a.lu = static_cast<float4*>(b->lu.p);
  a.le = static_cast<float2*>(b->le.p);
  a.tcount = static_cast<uint32_t*>(b->tcount.p);
  a.toff = static_cast<uint32_t*>(b->toff.p);
  a.tcur = static_cast<uint32_t*>(b->tcur.p);
  a.gt_ = static_cast<uint32_t*>(b->gl_t.p);
  a.gc = static_cast<uint32_t*>(b->gl_c.p);
  a.gu = static_cast<float4*>(b->gl_u.p);
  a.ge_ = static_cast<float2*>(b->gl_e.p);
  a.st = static_cast<uint32_t*>(b->st.p);
  a.sc = static_cast<uint32_t*>(b->sc.p);
  a.su = static_cast<float4*>(b->su.p);
  a.se = static_cast<float2*>(b->se.p);
  a.trip = static_cast<uint32_t*>(b->trip.p);
  a.ccount = static_cast<uint32_t*>(b->ccount.p);
  a.coff = static_cast<uint32_t*>(b->coff.p);
  a.ccur = static_cast<uint32_t*>(b->ccur.p);
  a.ut = static_cast<uint32_t*>(b->ut.p);
  a.ue = static_cast<float*>(b->ue.p);
  a.ucell = static_cast<uint32_t*>(b->ucell.p);
  a.gt = static_cast<uint32_t*>(b->gt.p);
  a.ge = static_cast<float*>(b->ge.p);
  a.max_cell = static_cast<uint32_t*>(b->max_cell_dev.p);
  const int64_t ncell = int64_t(a.G) * a.G;
  bbc_status st;
  if ((st = launch_fill_u32(a.tcount, 0, b->n_tuples, s))) return st;
  if ((st = launch_fill_u32(a.tcur, 0, b->n_tuples, s))) return st;
  if ((st = launch_fill_u32(a.ccount, 0, ncell, s))) return st;
  if ((st = launch_fill_u32(a.ccur, 0, ncell, s))) return st;
  if ((st = launch_fill_u32(a.max_cell, 0, 1, s))) return st;
  const unsigned gl = 2048;
  hipLaunchKernelGGL(k_leaf_count, dim3(gl), dim3(256), 0, s, a);
  if ((st = launch_scan_u32(a.tcount, a.toff, b->n_tuples, b->scan_tmp.p, s))) return st;
  hipLaunchKernelGGL(k_leaf_scatter, dim3(gl), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_leaf_rank, dim3(gl), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_grid_tuple, dim3(4096), dim3(kGridThreads), 0, s, a);
  if ((st = launch_scan_u32(a.ccount, a.coff, ncell, b->scan_tmp.p, s))) return st;
  hipLaunchKernelGGL(k_grid_scatter, dim3(gl), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_grid_rank, dim3(gl), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_tuple_records,
                     dim3(unsigned(std::max<int64_t>(1, std::min<int64_t>((b->n_tuples + 255) / 256, 4096)))),
                     dim3(256), 0, s, a, b->scene, static_cast<const float4*>(b->root.p), static_cast<float*>(b->trec.p),
                     b->rec_floats);
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

}  // namespace bbc
