// Bound storage (Sec. 6.1): group the leaves by tuple and splat every leaf's
// irradiance bound into the receiver-grid cells its closed position bound
// touches, keeping per (cell, tuple) the maximum (Eq. eq_pertuple_b, m = 1).
// The grid is a CSR: offsets per cell, then (tuple, E~) sorted by tuple.
//
// Kernels (all counts read from device memory, no host synchronisation):
//   k_leaf_count / scan / k_leaf_scatter / k_leaf_rank   leaves grouped by tuple
//   k_leaf_rects   cell rectangle of every leaf
//   k_grid_cells<false> / scan / k_grid_cells<true>      entries per cell, then
//                  the CSR, one workgroup per 16 x 16 tile of cells
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
  uint32_t leaf_cap, grid_cap;
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
  uint4* lrect;     // cell rectangle, tuple and E_hi bits of each sorted leaf
  uint32_t* lcoarse;  // rectangle in tiles of each sorted leaf (padded with empty ones)
  uint32_t* ccount;
  uint32_t* coff;
  uint32_t* gt;     // entries, sorted by tuple inside each cell, then the cover-all list
  float* ge;
  uint32_t* max_cell;
  // cover-all list: per-tuple flag (then its scan: the tuple's slot in the
  // list) and the largest E_hi of the tuple's leaves
  uint32_t* cflag;
  uint32_t* cpos;
  float* cE;
  double cover_cells;  // footprint (leaf-cell records) at which a tuple goes to the list; 0: never
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

// Union of the receiver bounds of each run of kLeafGroup sorted leaves (the
// last run may be shorter).  fminf / fmaxf take the non-NaN operand, so a leaf
// whose bound holds a target makes its run's union hold it too.
__global__ void k_leaf_groups(const float4* su, const BuildCounters* C, uint32_t n_host, uint32_t cap, float4* sug) {
  const uint32_t n = C ? min(C->n_leaves, cap) : n_host;
  const uint32_t ng = (n + kLeafGroup - 1) / kLeafGroup;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < ng; g += gridDim.x * blockDim.x) {
    float4 r = make_float4(INFINITY, -INFINITY, INFINITY, -INFINITY);
    const uint32_t e = min(n, (g + 1) * kLeafGroup);
    for (uint32_t i = g * kLeafGroup; i < e; ++i) {
      const float4 u = su[i];
      r.x = fminf(r.x, u.x);
      r.y = fmaxf(r.y, u.y);
      r.z = fminf(r.z, u.z);
      r.w = fmaxf(r.w, u.w);
    }
    sug[g] = r;
  }
}

bbc_status launch_leaf_groups(Bounds* b, const BuildCounters* counters, uint32_t n_host, hipStream_t s) {
  const size_t cap = counters ? b->leaf_cap : size_t(n_host);
  bbc_status e;
  if ((e = ensure(b->sug, (cap / kLeafGroup + 1) * 16, b))) return e;
  hipLaunchKernelGGL(k_leaf_groups, dim3(512), dim3(256), 0, s, static_cast<const float4*>(b->su.p), counters,
                     n_host, uint32_t(std::min<size_t>(cap, 0xffffffffu)), static_cast<float4*>(b->sug.p));
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

// ---------------------------------------------------------------- receiver grid
// Cell of a receiver coordinate: the product x G is exact in FP64 (24-bit
// significand times G <= 4096), so a bound's edge is never rounded into the
// next cell.
__device__ __forceinline__ int cell_of(float x, int G) {
  const double c = floor(double(fminf(fmaxf(x, 0.f), 1.f)) * double(G));  // NaN maps to 0
  return min(G - 1, max(0, int(c)));
}

// Cover-all decision per tuple (Sec. 6.1 bound storage, cover-all reading):
// the sum over its leaves of the number of cells of their closed cell
// rectangles, against cover_frac * G^2; and the largest E_hi of its leaves.
__global__ void k_tuple_cover(RecArgs a) {
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < a.n_tuples;
       t += int64_t(gridDim.x) * blockDim.x) {
    const uint32_t lb = a.toff[t], le = a.toff[t + 1];
    uint64_t cells = 0;
    float emax = 0.f;
    for (uint32_t i = lb; i < le; ++i) {
      const float4 u = a.su[i];
      cells += uint64_t(cell_of(u.y, a.G) - cell_of(u.x, a.G) + 1) * uint64_t(cell_of(u.w, a.G) - cell_of(u.z, a.G) + 1);
      emax = fmaxf(emax, a.se[i].y);
    }
    a.cflag[t] = (a.cover_cells > 0.0 && cells > 0 && double(cells) >= a.cover_cells) ? 1u : 0u;
    a.cE[t] = emax;
  }
}

// The cover-all list after the cells' entries: tuple t with its flag set goes
// to slot cpos[t] (tuples ascending), and the last offset closes the list.
__global__ void k_cover_write(RecArgs a) {
  const uint32_t G2 = uint32_t(a.G) * uint32_t(a.G);
  const uint32_t base = a.coff[G2], n_cover = a.cpos[a.n_tuples];
  if (uint64_t(base) + n_cover > a.grid_cap) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      atomicOr(&a.C->overflow, 4u);
      a.C->n_triples = base + n_cover;
    }
    return;
  }
  for (int64_t t = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; t < a.n_tuples;
       t += int64_t(gridDim.x) * blockDim.x)
    if (a.cflag[t]) {
      a.gt[base + a.cpos[t]] = uint32_t(t);
      a.ge[base + a.cpos[t]] = a.cE[t];
    }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.coff[G2 + 1] = base + n_cover;
    a.C->n_entries = base + n_cover;
    a.C->n_cover = n_cover;
    *a.max_cell += n_cover;  // every point reads its cell's list and the cover-all list
  }
}

// What the grid needs of every leaf (in the tuple order of the sorted
// leaves), in one 16-byte record: its closed cell rectangle packed as
// (cu0 | cu1 << 16, cv0 | cv1 << 16), its tuple, and the bits of its E_hi
// (E_hi >= 0, so the bit order is the value order); and, for the scan of the
// grid kernel, the rectangle in units of 16-cell tiles in one word
// (tu0 | tu1 << 8 | tv0 << 16 | tv1 << 24; grid_res <= 4096 keeps tile
// indices below 256).  Coarse words from the last leaf up to two scan steps
// beyond it hold an empty rectangle (tu0 = 255 > tu1 = 0).
constexpr int kCellTile = 16, kCellThreads = kCellTile * kCellTile;
constexpr int kPerThread = 8, kChunk = kCellThreads * kPerThread;  // leaves tested per scan step
constexpr uint32_t kEmptyCoarse = 0x000000ffu;

__global__ void k_leaf_rects(RecArgs a) {
  const uint32_t n = min(a.C->n_leaves, a.leaf_cap);
  const uint32_t n_pad = (n + uint32_t(kChunk) - 1) / uint32_t(kChunk) * uint32_t(kChunk) + uint32_t(kChunk);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n_pad; i += gridDim.x * blockDim.x) {
    if (i >= n) {
      a.lcoarse[i] = kEmptyCoarse;
      continue;
    }
    if (a.cflag[a.st[i]]) {  // the tuple is in the cover-all list: the leaf meets no tile
      a.lcoarse[i] = kEmptyCoarse;
      continue;
    }
    const float4 u = a.su[i];
    const uint32_t cu0 = uint32_t(cell_of(u.x, a.G)), cu1 = uint32_t(cell_of(u.y, a.G));
    const uint32_t cv0 = uint32_t(cell_of(u.z, a.G)), cv1 = uint32_t(cell_of(u.w, a.G));
    a.lrect[i] = make_uint4(cu0 | cu1 << 16, cv0 | cv1 << 16, a.st[i], __float_as_uint(a.se[i].y));
    a.lcoarse[i] = (cu0 / kCellTile) | (cu1 / kCellTile) << 8 | (cv0 / kCellTile) << 16 | (cv1 / kCellTile) << 24;
  }
}

// Cell-major rasterisation.  One workgroup per tile of 16 x 16 cells, one
// thread per cell.  The workgroup scans all leaves in their tuple order,
// keeps those whose rectangle meets the tile (in order, in LDS), and each
// thread walks that list: consecutive leaves of one tuple that touch its cell
// merge into one entry with the maximum E_hi, and a new tuple closes the
// previous entry.  Each cell's list therefore comes out sorted by tuple, with
// no atomics on cells and no sort.  WRITE = false counts the entries per cell
// (and the largest cell); WRITE = true writes them at the scanned offsets.
constexpr int kLeafBuf = kChunk + 1024;  // leaves meeting the tile, staged per flush
constexpr uint32_t kNoRect = 0u;

// Bits lo..hi of a 16-bit mask (empty when lo > hi).
__device__ __forceinline__ uint32_t span_mask(int lo, int hi) {
  return lo > hi ? 0u : ((0xffffu >> (15 - hi)) & (0xffffu << lo));
}
constexpr uint32_t kNoTuple = 0xffffffffu;

template <bool WRITE>
__global__ void __launch_bounds__(kCellThreads) k_grid_cells(RecArgs a) {
  __shared__ __align__(16) uint32_t s_t[kLeafBuf + 4], s_key[kLeafBuf + 4], s_rect[kLeafBuf + 4];
  // s_t holds the leaf index until the staged leaves are resolved before a walk
  const int G = a.G, tid = int(threadIdx.x), lane = tid % BBC_WAVE;
  const uint32_t n = min(a.C->n_leaves, a.leaf_cap);
  const int nt = (G + kCellTile - 1) / kCellTile;
  const uint32_t total = WRITE ? a.coff[uint32_t(G) * uint32_t(G)] : 0u;
  if (WRITE && total > a.grid_cap) {
    if (blockIdx.x == 0 && tid == 0) {
      atomicOr(&a.C->overflow, 4u);
      a.C->n_triples = total;
    }
    return;
  }
  uint32_t mx = 0;
  for (int tile = blockIdx.x; tile < nt * nt; tile += gridDim.x) {
    const int tu0 = (tile / nt) * kCellTile, tv0 = (tile % nt) * kCellTile;
    const int lu = tid / kCellTile, lv = tid % kCellTile;
    const int cu = tu0 + lu, cv = tv0 + lv;
    const bool inside = cu < G && cv < G;
    const uint32_t cell = uint32_t(cu) * uint32_t(G) + uint32_t(cv);
    uint32_t p = (WRITE && inside) ? a.coff[cell] : 0u;
    uint32_t cnt = 0, last_t = kNoTuple, last_key = 0u;
    uint32_t nb = 0;  // leaves staged in LDS (the same in every thread)
    // the leaf's cell rectangle inside the tile as two 16-bit masks (rows in
    // the low half, columns in the high half); this cell's bits:
    const uint32_t bu = 1u << lu, bv = 1u << (16 + lv);
    auto visit = [&](uint32_t t, uint32_t key) {
      if (t == last_t) {
        last_key = max(last_key, key);
        return;
      }
      if (last_t != kNoTuple) {
        if (WRITE) {
          a.gt[p] = last_t;
          a.ge[p] = __uint_as_float(last_key);
          ++p;
        }
        ++cnt;
      }
      last_t = t;
      last_key = key;
    };
    // four staged leaves per step (the list is padded with empty masks); the
    // staged leaf indices are first replaced by the leaves' tuples, E_hi bits
    // and rectangle masks (one load per staged leaf, spread over the block)
    auto walk = [&]() {
      for (uint32_t i = uint32_t(tid); i < nb; i += kCellThreads) {
        const uint4 r = a.lrect[s_t[i]];
        const int u0 = int(r.x & 0xffffu), u1 = int(r.x >> 16), v0 = int(r.y & 0xffffu), v1 = int(r.y >> 16);
        s_rect[i] = span_mask(max(u0 - tu0, 0), min(u1 - tu0, kCellTile - 1)) |
                    span_mask(max(v0 - tv0, 0), min(v1 - tv0, kCellTile - 1)) << 16;
        s_t[i] = r.z;
        s_key[i] = r.w;
      }
      if (tid < 4) s_rect[nb + tid] = kNoRect;  // pad to a multiple of four
      __syncthreads();
      if (!inside) return;
      for (uint32_t i = 0; i < nb; i += 4) {
        const uint4 m = *reinterpret_cast<const uint4*>(&s_rect[i]);
        const bool h0 = (m.x & bu) && (m.x & bv), h1 = (m.y & bu) && (m.y & bv);
        const bool h2 = (m.z & bu) && (m.z & bv), h3 = (m.w & bu) && (m.w & bv);
        if (!(h0 || h1 || h2 || h3)) continue;
        const uint4 t = *reinterpret_cast<const uint4*>(&s_t[i]);
        const uint4 k = *reinterpret_cast<const uint4*>(&s_key[i]);
        if (h0) visit(t.x, k.x);
        if (h1) visit(t.y, k.y);
        if (h2) visit(t.z, k.z);
        if (h3) visit(t.w, k.w);
      }
    };
    // Leaves are tested kChunk at a time on their coarse words, kPerThread
    // consecutive ones per thread, so that one block scan orders the hits;
    // the next step's words are loaded while the current ones are tested (two
    // register buffers in turn).  Only the indices of hits are staged.
    const uint32_t ti = uint32_t(tu0 / kCellTile), tj = uint32_t(tv0 / kCellTile);
    const uint4* coarse4 = reinterpret_cast<const uint4*>(a.lcoarse);
    uint4 ra[kPerThread / 4], rb[kPerThread / 4];
    auto load = [&](uint4* r, uint32_t base) {
#pragma unroll
      for (int c = 0; c < kPerThread / 4; ++c) r[c] = coarse4[(base + uint32_t(tid * kPerThread)) / 4 + c];
    };
    auto test = [&](const uint4* r, uint32_t base) {
      if (base >= n) return;
      uint32_t hitmask = 0;
#pragma unroll
      for (int c = 0; c < kPerThread; ++c) {
        const uint32_t w = c % 4 == 0 ? r[c / 4].x : c % 4 == 1 ? r[c / 4].y : c % 4 == 2 ? r[c / 4].z : r[c / 4].w;
        const bool hit = (w & 0xffu) <= ti && ((w >> 8) & 0xffu) >= ti && ((w >> 16) & 0xffu) <= tj && (w >> 24) >= tj;
        hitmask |= hit ? 1u << c : 0u;
      }
      if (!__syncthreads_or(int(hitmask))) return;
      uint32_t tot;
      uint32_t q = nb + block_exclusive_scan(uint32_t(__popc(hitmask)), &tot);
#pragma unroll
      for (int c = 0; c < kPerThread; ++c)
        if (hitmask & (1u << c)) s_t[q++] = base + uint32_t(tid * kPerThread + c);
      nb += tot;
      __syncthreads();
      if (nb > uint32_t(kLeafBuf - kChunk)) {
        walk();
        nb = 0;
        __syncthreads();
      }
    };
    load(ra, 0u);
    for (uint32_t k0 = 0; k0 < n; k0 += 2 * kChunk) {
      load(rb, k0 + kChunk);
      test(ra, k0);
      load(ra, k0 + 2 * kChunk);
      test(rb, k0 + kChunk);
    }
    walk();
    if (inside) {
      if (last_t != kNoTuple) {
        if (WRITE) {
          a.gt[p] = last_t;
          a.ge[p] = __uint_as_float(last_key);
        }
        ++cnt;
      }
      if (!WRITE) a.ccount[cell] = cnt;
    }
    mx = max(mx, cnt);
    __syncthreads();
  }
  if (!WRITE) {
    mx = wave_max(mx);
    if (lane == 0 && mx) atomicMax(a.max_cell, mx);
  }
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
  a.grid_cap = uint32_t(b->grid_cap);
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
  a.lrect = static_cast<uint4*>(b->lrect.p);
  a.lcoarse = static_cast<uint32_t*>(b->lcoarse.p);
  a.ccount = static_cast<uint32_t*>(b->ccount.p);
  a.coff = static_cast<uint32_t*>(b->coff.p);
  a.gt = static_cast<uint32_t*>(b->gt.p);
  a.ge = static_cast<float*>(b->ge.p);
  a.max_cell = static_cast<uint32_t*>(b->max_cell_dev.p);
  a.cflag = static_cast<uint32_t*>(b->cflag.p);
  a.cpos = static_cast<uint32_t*>(b->cpos.p);
  a.cE = static_cast<float*>(b->cE.p);
  a.cover_cells = double(b->params.cover_frac) * double(a.G) * double(a.G);
  const int64_t ncell = int64_t(a.G) * a.G;
  bbc_status st;
  if ((st = launch_fill_u32(a.tcount, 0, b->n_tuples, s))) return st;
  if ((st = launch_fill_u32(a.tcur, 0, b->n_tuples, s))) return st;
  if ((st = launch_fill_u32(a.max_cell, 0, 1, s))) return st;
  const unsigned gl = 2048;
  hipLaunchKernelGGL(k_leaf_count, dim3(gl), dim3(256), 0, s, a);
  if ((st = launch_scan_u32(a.tcount, a.toff, b->n_tuples, b->scan_tmp.p, s))) return st;
  hipLaunchKernelGGL(k_leaf_scatter, dim3(gl), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_leaf_rank, dim3(gl), dim3(256), 0, s, a);
  if ((st = launch_leaf_groups(b, a.C, 0, s))) return st;
  const unsigned gt_ = unsigned(std::max<int64_t>(1, std::min<int64_t>((b->n_tuples + 255) / 256, 4096)));
  hipLaunchKernelGGL(k_tuple_cover, dim3(gt_), dim3(256), 0, s, a);
  if ((st = launch_scan_u32(a.cflag, a.cpos, b->n_tuples, b->scan_tmp.p, s))) return st;
  hipLaunchKernelGGL(k_leaf_rects, dim3(gl), dim3(256), 0, s, a);
  const int nt = (a.G + kCellTile - 1) / kCellTile;
  const unsigned gc = unsigned(nt) * unsigned(nt);
  hipLaunchKernelGGL(k_grid_cells<false>, dim3(gc), dim3(kCellThreads), 0, s, a);
  if ((st = launch_scan_u32(a.ccount, a.coff, ncell, b->scan_tmp.p, s))) return st;
  hipLaunchKernelGGL(k_grid_cells<true>, dim3(gc), dim3(kCellThreads), 0, s, a);
  hipLaunchKernelGGL(k_cover_write, dim3(gt_), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_tuple_records,
                     dim3(unsigned(std::max<int64_t>(1, std::min<int64_t>((b->n_tuples + 255) / 256, 4096)))),
                     dim3(256), 0, s, a, b->scene, static_cast<const float4*>(b->root.p), static_cast<float*>(b->trec.p),
                     b->rec_floats);
  BBC_HIP(hipGetLastError());
  return BBC_OK;
}

}  // namespace bbc
