// Host side of the C ABI (include/bbc.h): argument validation, library-owned
// device buffers, capacity regrowth, and the stage launch sequences.
#include <cmath>
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace bbc {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

bbc_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? BBC_ENOMEM : BBC_EDEVICE;
}

void release_graph(QueryGraph& g) {
  if (g.stream) (void)hipStreamSynchronize(g.stream);
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.in) (void)hipEventDestroy(g.in);
  if (g.out) (void)hipEventDestroy(g.out);
  if (g.stream) (void)hipStreamDestroy(g.stream);
  g = QueryGraph{};
}

static bbc_status invalid(const char* msg) {
  set_error(msg);
  return BBC_EINVAL;
}

bbc_status ensure(DevBuf& b, size_t bytes, Bounds* owner) {
  if (bytes == 0) bytes = 4;
  if (b.bytes >= bytes) return BBC_OK;
  if (b.p) {
    BBC_HIP(hipFree(b.p));
    if (owner) owner->device_bytes -= int64_t(b.bytes);
    b.p = nullptr;
    b.bytes = 0;
  }
  void* p = nullptr;
  const hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    set_error("device allocation of " + std::to_string(bytes) + " bytes failed");
    return BBC_ENOMEM;
  }
  b.p = p;
  b.bytes = bytes;
  if (owner) owner->device_bytes += int64_t(bytes);
  return BBC_OK;
}

void release(DevBuf& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

static void release_all(Bounds* b) {
  DevBuf* all[] = {&b->pos, &b->nrm, &b->epos, &b->eI, &b->eedge, &b->counters, &b->root, &b->init_q, &b->l0f_q, &b->q[0],
                   &b->q[1], &b->fq, &b->lt, &b->lc, &b->lu, &b->le, &b->gl_t, &b->gl_c, &b->gl_u, &b->gl_e, &b->st, &b->sc, &b->su, &b->sug, &b->se, &b->tcount,
                   &b->toff, &b->tcur, &b->lrect, &b->lcoarse, &b->ccount, &b->coff, &b->gt, &b->ge,
                   &b->scan_tmp, &b->trec, &b->pos2, &b->nrm2, &b->box2, &b->rowcount, &b->rowoff, &b->tid,
                   &b->qw_buf, &b->max_cell_dev, &b->qcounters, &b->cflag, &b->cpos, &b->cE, &b->red_tab,
                   &b->srec[0], &b->srec[1]};
  for (DevBuf* d : all) release(*d);
  b->red_ready = false;
  b->srec_cap = 0;
  b->device_bytes = 0;
}

static bbc_status copy_in(DevBuf& dst, const void* src, size_t bytes, int memory, Bounds* owner, hipStream_t s) {
  bbc_status e = ensure(dst, bytes, owner);
  if (e) return e;
  BBC_HIP(hipMemcpyAsync(dst.p, src, bytes, memory == BBC_MEM_DEVICE ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         s));
  return BBC_OK;
}

static bbc_status validate(const bbc_scene* sc, const bbc_emitters* em, const bbc_subdiv_params* p) {
  if (!sc || !em || !p) return invalid("null scene, emitters or params");
  if (sc->chain != BBC_CHAIN_R && sc->chain != BBC_CHAIN_T && sc->chain != BBC_CHAIN_RR)
    return invalid("unknown chain type");
  if (sc->chain == BBC_CHAIN_RR) {
    if (sc->n_tri2 < 1 || !sc->pos2 || !sc->nrm2) return invalid("two reflections need n_tri2 >= 1 and pos2/nrm2");
    if (double(sc->n_tri) * double(sc->n_tri2) * double(em->n) > 4294967000.0)
      return invalid("more than 2^32 triangle pairs");
  }
  if (sc->memory != BBC_MEM_HOST && sc->memory != BBC_MEM_DEVICE) return invalid("scene memory flag");
  if (em->memory != BBC_MEM_HOST && em->memory != BBC_MEM_DEVICE) return invalid("emitter memory flag");
  if (sc->n_tri < 1 || !sc->pos || !sc->nrm) return invalid("scene needs n_tri >= 1 and pos/nrm arrays");
  if (em->n < 1 || !em->pos || !em->I0) return invalid("emitters need n >= 1 and pos/I0 arrays");
  if (double(sc->n_tri) * double(em->n) > 4294967000.0) return invalid("more than 2^32 tuples");
  if (em->edges && sc->chain != BBC_CHAIN_R) return invalid("area lights (edges) need the single-reflection chain");
  const double f1[3] = {sc->f1[0], sc->f1[1], sc->f1[2]}, f2[3] = {sc->f2[0], sc->f2[1], sc->f2[2]};
  const double c[3] = {f1[1] * f2[2] - f1[2] * f2[1], f1[2] * f2[0] - f1[0] * f2[2], f1[0] * f2[1] - f1[1] * f2[0]};
  const double ak = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  if (!(ak > 0.0) || !std::isfinite(ak)) return invalid("degenerate receiver (|f1 x f2| = 0)");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(sc->q0[k])) return invalid("receiver origin not finite");
  if (sc->chain == BBC_CHAIN_T && !(sc->eta > 0.f && std::isfinite(sc->eta))) return invalid("eta must be > 0");
  if (p->max_depth < 0 || p->max_depth > kMaxDepth) return invalid("max_depth must be in [0, 14]");
  if (!(p->sigma >= 0.f) || !(p->alpha >= 1.f)) return invalid("sigma >= 0 and alpha >= 1 required");
  if (p->grid_res < 1 || p->grid_res > 4096) return invalid("grid_res must be in [1, 4096]");
  if (p->init_pieces < 1 || p->init_pieces > 256) return invalid("init_pieces must be in [1, 256]");
  if (p->init_levels < 0 || p->init_levels > 12) return invalid("init_levels must be in [0, 12]");
  if (p->flags & ~(BBC_FLAG_FIXED_DEPTH | BBC_FLAG_NO_REMAINDER | BBC_FLAG_IMPLICIT_IRR | BBC_FLAG_DEGREE_REDUCTION))
    return invalid("unknown flags");
  if (!(p->cover_frac >= 0.f) || !std::isfinite(p->cover_frac)) return invalid("cover_frac must be finite and >= 0");
  return BBC_OK;
}

static bbc_status construct_pairs(Bounds* b, hipStream_t s);

static bbc_status run_build(Bounds* b, hipStream_t s) {
  const int64_t G = b->params.grid_res;
  const int64_t ncell = G * G;
  bbc_status e;
  if (b->scene.chain == BBC_CHAIN_RR && (e = construct_pairs(b, s))) return e;
  if (b->q_cap == 0) {
    b->q_cap = size_t(std::max<int64_t>(4 * b->n_tuples, 1 << 20));
    b->fq_cap = b->q_cap;
    b->leaf_cap = b->q_cap;
    b->grid_cap = size_t(32) << 20;
  }
  for (int attempt = 0; attempt < 5; ++attempt) {
    if ((e = ensure(b->counters, sizeof(BuildCounters), b)) || (e = ensure(b->root, b->n_tuples * 16, b)) ||
        (e = ensure(b->init_q, b->n_tuples * 4, b)) || (e = ensure(b->l0f_q, b->n_tuples * 4, b)) ||
        (e = ensure(b->q[0], b->q_cap * 8, b)) || (e = ensure(b->q[1], b->q_cap * 8, b)) ||
        (e = ensure(b->fq, b->fq_cap * 8, b)) || (e = ensure(b->lt, b->leaf_cap * 4, b)) ||
        (e = ensure(b->lc, b->leaf_cap * 4, b)) || (e = ensure(b->lu, b->leaf_cap * 16, b)) ||
        (e = ensure(b->le, b->leaf_cap * 8, b)) || (e = ensure(b->gl_t, b->leaf_cap * 4, b)) ||
        (e = ensure(b->gl_c, b->leaf_cap * 4, b)) || (e = ensure(b->gl_u, b->leaf_cap * 16, b)) ||
        (e = ensure(b->gl_e, b->leaf_cap * 8, b)) || (e = ensure(b->st, b->leaf_cap * 4, b)) ||
        (e = ensure(b->sc, b->leaf_cap * 4, b)) || (e = ensure(b->su, b->leaf_cap * 16, b)) ||
        (e = ensure(b->se, b->leaf_cap * 8, b)) || (e = ensure(b->tcount, b->n_tuples * 4, b)) ||
        (e = ensure(b->toff, (b->n_tuples + 1) * 4, b)) || (e = ensure(b->tcur, b->n_tuples * 4, b)) ||
        (e = ensure(b->lrect, b->leaf_cap * 16, b)) || (e = ensure(b->lcoarse, (b->leaf_cap + 3 * 2048) * 4, b)) || (e = ensure(b->ccount, ncell * 4, b)) ||
        (e = ensure(b->coff, (ncell + 2) * 4, b)) || (e = ensure(b->gt, b->grid_cap * 4, b)) ||
        (e = ensure(b->cflag, b->n_tuples * 4, b)) || (e = ensure(b->cpos, (b->n_tuples + 1) * 4, b)) ||
        (e = ensure(b->cE, b->n_tuples * 4, b)) ||
        (e = ensure(b->ge, b->grid_cap * 4, b)) ||
        (e = ensure(b->scan_tmp, scan_tmp_bytes(std::max(ncell, b->n_tuples)) + 64, b)) ||
        (e = ensure(b->trec, size_t(std::max<int64_t>(b->n_tuples, 1)) * b->rec_floats * 4, b)) ||
        (e = ensure(b->max_cell_dev, 64, b)))
      return e;
    if ((e = launch_build(b, s))) return e;
    if ((e = launch_record(b, s))) return e;
    BBC_HIP(hipMemcpyAsync(&b->host, b->counters.p, sizeof(BuildCounters), hipMemcpyDeviceToHost, s));
    uint32_t mc = 0;
    BBC_HIP(hipMemcpyAsync(&mc, b->max_cell_dev.p, 4, hipMemcpyDeviceToHost, s));
    BBC_HIP(hipStreamSynchronize(s));
    const uint32_t ov = b->host.overflow;
    if (!ov) {
      b->n_leaves = b->host.n_leaves;
      b->n_entries = b->host.n_entries;
      b->max_cell = mc;
      return BBC_OK;
    }
    if (ov & (1u | 2u | 8u)) {
      b->q_cap *= 4;
      b->fq_cap *= 4;
      b->leaf_cap *= 4;
    }
    if (ov & 4u) b->grid_cap = std::max<size_t>(b->grid_cap * 2, size_t(b->host.n_triples) + 1024);
    if (ov & 32u) {  // a depth had more items than subdivision records: room for the most seen, and more
      size_t need = 4 * size_t(b->srec_cap);
      for (uint32_t c : b->host.qcount) need = std::max<size_t>(need, c);
      b->srec_cap = uint32_t(std::min(need + 3, b->q_cap)) & ~3u;
    }
    if (b->q_cap > (size_t(1) << 31) || b->grid_cap > (size_t(1) << 31)) break;
  }
  const uint32_t ov = b->host.overflow;
  std::string what;
  if (ov & 1u) what += " subdivision queue;";
  if (ov & 2u) what += " leaves;";
  if (ov & 4u) what += " grid entries (" + std::to_string(b->host.n_triples) + " cell-tuple pairs);";
  if (ov & 8u) what += " FP64 queue;";
  if (ov & 16u) what += " domain initialisation;";
  if (ov & 32u) what += " subdivision records;";
  set_error("device work queues overflowed their maximum capacity:" + what);
  return BBC_EQUEUE;
}

static bbc_status load_scene(Bounds* b, const bbc_scene* sc, const bbc_emitters* em, const bbc_subdiv_params* p,
                             hipStream_t s) {
  bbc_status e;
  const size_t nt = size_t(sc->n_tri);
  if ((e = copy_in(b->pos, sc->pos, nt * 9 * 4, sc->memory, b, s))) return e;
  if ((e = copy_in(b->nrm, sc->nrm, nt * 9 * 4, sc->memory, b, s))) return e;
  if ((e = copy_in(b->epos, em->pos, size_t(em->n) * 3 * 4, em->memory, b, s))) return e;
  if ((e = copy_in(b->eI, em->I0, size_t(em->n) * 4, em->memory, b, s))) return e;
  if (em->edges && (e = copy_in(b->eedge, em->edges, size_t(em->n) * 6 * 4, em->memory, b, s))) return e;
  if (sc->chain == BBC_CHAIN_RR) {
    const size_t n2 = size_t(sc->n_tri2);
    if ((e = copy_in(b->pos2, sc->pos2, n2 * 9 * 4, sc->memory, b, s))) return e;
    if ((e = copy_in(b->nrm2, sc->nrm2, n2 * 9 * 4, sc->memory, b, s))) return e;
  }
  b->params = *p;
  DevScene& d = b->scene;
  d.chain = sc->chain;
  d.n_tri = sc->n_tri;
  d.pos = static_cast<const float*>(b->pos.p);
  d.nrm = static_cast<const float*>(b->nrm.p);
  d.n_emit = em->n;
  d.epos = static_cast<const float*>(b->epos.p);
  d.eI = static_cast<const float*>(b->eI.p);
  d.eedge = em->edges ? static_cast<const float*>(b->eedge.p) : nullptr;
  d.eta = sc->chain == BBC_CHAIN_T ? sc->eta : 1.f;
  for (int k = 0; k < 3; ++k) {
    d.q0[k] = sc->q0[k];
    d.f1[k] = sc->f1[k];
    d.f2[k] = sc->f2[k];
  }
  d.n_tri2 = sc->chain == BBC_CHAIN_RR ? sc->n_tri2 : 0;
  d.pos2 = sc->chain == BBC_CHAIN_RR ? static_cast<const float*>(b->pos2.p) : nullptr;
  d.nrm2 = sc->chain == BBC_CHAIN_RR ? static_cast<const float*>(b->nrm2.p) : nullptr;
  d.tid = nullptr;
  b->n_dense = sc->n_tri * em->n * (sc->chain == BBC_CHAIN_RR ? sc->n_tri2 : 1);
  b->n_tuples = sc->n_tri * em->n;
  b->rec_floats = sc->chain == BBC_CHAIN_RR ? kRecFloatsRR : kRecFloats;
  return BBC_OK;
}

// Tuple construction for two reflections: count the candidate pairs of every
// (emitter, first triangle) row, scan, read the total (one host
// synchronisation: it sizes every per-tuple buffer), and write the pairs.
static bbc_status construct_pairs(Bounds* b, hipStream_t s) {
  DevScene& d = b->scene;
  const int64_t rows = d.n_emit * d.n_tri;
  bbc_status e;
  if ((e = ensure(b->box2, size_t(d.n_tri2) * 6 * 8, b)) || (e = ensure(b->rowcount, size_t(rows) * 4, b)) ||
      (e = ensure(b->rowoff, size_t(rows + 1) * 4 + 8, b)) || (e = ensure(b->scan_tmp, scan_tmp_bytes(rows) + 64, b)))
    return e;
  double* box2 = static_cast<double*>(b->box2.p);
  uint32_t* rc = static_cast<uint32_t*>(b->rowcount.p);
  uint32_t* ro = static_cast<uint32_t*>(b->rowoff.p);
  if ((e = launch_pairs(d, box2, rc, ro, nullptr, false, s))) return e;
  if ((e = launch_scan_u32(rc, ro, rows, b->scan_tmp.p, s))) return e;
  uint32_t total = 0;
  BBC_HIP(hipMemcpyAsync(&total, ro + rows, 4, hipMemcpyDeviceToHost, s));
  BBC_HIP(hipStreamSynchronize(s));
  if ((e = ensure(b->tid, size_t(std::max<uint32_t>(total, 1)) * 4, b))) return e;
  d.tid = static_cast<const uint32_t*>(b->tid.p);
  if (total && (e = launch_pairs(d, box2, rc, ro, static_cast<uint32_t*>(b->tid.p), true, s))) return e;
  b->n_tuples = total;
  if (b->tuples_cap < total) {  // per-tuple buffers are sized by the tuple count
    b->q_cap = 0;
    b->tuples_cap = total;
  }
  return BBC_OK;
}

static hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }

// ---- bound file (bbc_bounds_save / bbc_bounds_load) ----
// Layout: FileHeader, then one section per array (u64 byte count, bytes) in
// the order of bound_sections(), then a u64 FNV-1a hash of every byte before it.
constexpr char kFileMagic[8] = {'B', 'B', 'C', 'B', 'O', 'U', 'N', 'D'};
constexpr uint32_t kFileVersion = 2;

struct FileHeader {
  char magic[8];
  uint32_t version;
  uint32_t header_bytes;
  int32_t chain, has_edges, rec_floats;
  float eta;
  int64_t n_tri, n_tri2, n_emit, n_tuples, n_dense, n_leaves, n_entries, max_cell;
  float q0[3], f1[3], f2[3];
  uint32_t pad;
  bbc_subdiv_params params;
  BuildCounters host;
};

struct Section {
  DevBuf* buf;
  size_t bytes;
};

// Every array a loaded handle needs for queries, exports and statistics.
static std::vector<Section> bound_sections(Bounds* b, int64_t n_tri, int64_t n_tri2, int64_t n_emit, bool edges) {
  const size_t nt = size_t(b->n_tuples), nl = size_t(b->n_leaves), ne = size_t(b->n_entries);
  const size_t G = size_t(b->params.grid_res);
  std::vector<Section> v = {{&b->pos, size_t(n_tri) * 36}, {&b->nrm, size_t(n_tri) * 36},
                            {&b->epos, size_t(n_emit) * 12}, {&b->eI, size_t(n_emit) * 4}};
  if (edges) v.push_back({&b->eedge, size_t(n_emit) * 24});
  if (b->scene.chain == BBC_CHAIN_RR) {
    v.push_back({&b->pos2, size_t(n_tri2) * 36});
    v.push_back({&b->nrm2, size_t(n_tri2) * 36});
    v.push_back({&b->tid, nt * 4});
  }
  const Section rest[] = {{&b->trec, nt * size_t(b->rec_floats) * 4},
                          {&b->root, nt * 16},
                          {&b->toff, (nt + 1) * 4},
                          {&b->st, nl * 4},
                          {&b->sc, nl * 4},
                          {&b->su, nl * 16},
                          {&b->se, nl * 8},
                          {&b->coff, (G * G + 2) * 4},
                          {&b->gt, ne * 4},
                          {&b->ge, ne * 4}};
  v.insert(v.end(), std::begin(rest), std::end(rest));
  return v;
}

struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void* p, size_t n) {
    const unsigned char* c = static_cast<const unsigned char*>(p);
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
};

// Host-side consistency of a loaded file: every index the query kernels
// follow (tuple offsets, grid offsets, tuple numbers, pair numbers, box codes)
// stays inside its array, so a damaged file cannot send a kernel out of bounds.
static bbc_status check_loaded(const FileHeader& fh, const std::vector<std::vector<char>>& data,
                               const std::vector<Section>& secs, const Bounds* b) {
  auto find = [&](const DevBuf* d) -> const std::vector<char>& {
    for (size_t i = 0; i < secs.size(); ++i)
      if (secs[i].buf == d) return data[i];
    return data[0];
  };
  const uint32_t* toff = reinterpret_cast<const uint32_t*>(find(&b->toff).data());
  const uint32_t* coff = reinterpret_cast<const uint32_t*>(find(&b->coff).data());
  const uint32_t* st = reinterpret_cast<const uint32_t*>(find(&b->st).data());
  const uint32_t* sc = reinterpret_cast<const uint32_t*>(find(&b->sc).data());
  const uint32_t* gt = reinterpret_cast<const uint32_t*>(find(&b->gt).data());
  const int64_t nt = fh.n_tuples, nl = fh.n_leaves, ne = fh.n_entries;
  const int64_t nc = int64_t(fh.params.grid_res) * fh.params.grid_res;
  if (toff[0] != 0 || int64_t(toff[nt]) != nl) return invalid("bound file: tuple offsets do not span the leaves");
  for (int64_t t = 0; t < nt; ++t)
    if (toff[t + 1] < toff[t]) return invalid("bound file: tuple offsets decrease");
  for (int64_t i = 0; i < nl; ++i) {
    if (int64_t(st[i]) >= nt || i < int64_t(toff[st[i]]) || i >= int64_t(toff[st[i] + 1]))
      return invalid("bound file: leaf tuple outside its offsets");
    const uint32_t depth = sc[i] >> 28, iu = (sc[i] >> kCodeBits) & ((1u << kCodeBits) - 1),
                   iv = sc[i] & ((1u << kCodeBits) - 1);
    if (depth > uint32_t(kMaxDepth) || iu >> depth || iv >> depth) return invalid("bound file: leaf code out of range");
  }
  int64_t mc = 0;
  // cells 0 .. nc-1, then the cover-all list as slice nc
  if (coff[0] != 0 || int64_t(coff[nc + 1]) != ne) return invalid("bound file: cell offsets do not span the entries");
  for (int64_t c = 0; c <= nc; ++c) {
    if (coff[c + 1] < coff[c]) return invalid("bound file: cell offsets decrease");
    if (c < nc) mc = std::max<int64_t>(mc, coff[c + 1] - coff[c]);
  }
  if (int64_t(coff[nc + 1] - coff[nc]) != int64_t(fh.host.n_cover))
    return invalid("bound file: cover-all list length differs from the header");
  if (mc + int64_t(fh.host.n_cover) != fh.max_cell) return invalid("bound file: fullest cell differs from the header");
  for (int64_t i = 0; i < ne; ++i)
    if (int64_t(gt[i]) >= nt) return invalid("bound file: grid entry names a tuple out of range");
  if (fh.chain == BBC_CHAIN_RR) {
    const uint32_t* tid = reinterpret_cast<const uint32_t*>(find(&b->tid).data());
    for (int64_t t = 0; t < nt; ++t)
      if (int64_t(tid[t]) >= fh.n_dense) return invalid("bound file: pair number out of range");
  }
  return BBC_OK;
}

static bbc_status read_exact(FILE* f, void* p, size_t n, Fnv& h) {
  if (n && std::fread(p, 1, n, f) != n) return invalid("bound file truncated");
  h.add(p, n);
  return BBC_OK;
}

static bbc_status load_file(FILE* f, Bounds* b, hipStream_t s) {
  Fnv h;
  FileHeader fh{};
  bbc_status e;
  if ((e = read_exact(f, &fh, sizeof fh, h))) return e;
  if (std::memcmp(fh.magic, kFileMagic, 8) != 0) return invalid("not a bound file (magic)");
  if (fh.version != kFileVersion || fh.header_bytes != sizeof(FileHeader))
    return invalid("bound file version or header size not supported");
  const bool rr = fh.chain == BBC_CHAIN_RR;
  if (fh.chain != BBC_CHAIN_R && fh.chain != BBC_CHAIN_T && !rr) return invalid("bound file: unknown chain");
  if (fh.params.grid_res < 1 || fh.params.grid_res > 4096 || fh.n_tri < 1 || fh.n_emit < 1 || fh.n_tuples < 0 ||
      fh.n_leaves < 0 || fh.n_entries < 0 || fh.n_leaves > (int64_t(1) << 32) || fh.n_entries > (int64_t(1) << 32) ||
      fh.max_cell < 0 || (rr && fh.n_tri2 < 1) || (!rr && fh.n_tri2 != 0) || (fh.has_edges && fh.chain != BBC_CHAIN_R))
    return invalid("bound file: counts out of range");
  const int64_t dense = fh.n_tri * fh.n_emit * (rr ? fh.n_tri2 : 1);
  if (double(fh.n_tri) * double(fh.n_emit) * double(rr ? fh.n_tri2 : 1) > 4294967000.0 || fh.n_dense != dense ||
      fh.n_tuples > dense || (!rr && fh.n_tuples != dense) || fh.rec_floats != (rr ? kRecFloatsRR : kRecFloats))
    return invalid("bound file: tuple counts inconsistent");
  b->params = fh.params;
  b->scene.chain = fh.chain;
  b->n_tuples = fh.n_tuples;
  b->n_dense = fh.n_dense;
  b->tuples_cap = rr ? fh.n_tuples : 0;
  b->rec_floats = fh.rec_floats;
  b->n_leaves = fh.n_leaves;
  b->n_entries = fh.n_entries;
  const std::vector<Section> secs = bound_sections(b, fh.n_tri, fh.n_tri2, fh.n_emit, fh.has_edges != 0);
  // The whole file's size follows from the header: check it before any
  // allocation, so that a damaged count cannot ask for a huge buffer.
  uint64_t want = sizeof(FileHeader) + 8;
  for (const Section& sec : secs) want += 8 + sec.bytes;
  const long here = std::ftell(f);
  if (here < 0 || std::fseek(f, 0, SEEK_END) != 0) return invalid("bound file is not seekable");
  const long end = std::ftell(f);
  if (end < 0 || std::fseek(f, here, SEEK_SET) != 0) return invalid("bound file is not seekable");
  if (uint64_t(end) != want) return invalid("bound file size differs from what its header describes");
  std::vector<std::vector<char>> data(secs.size());
  for (size_t i = 0; i < secs.size(); ++i) {
    uint64_t n = 0;
    if ((e = read_exact(f, &n, 8, h))) return e;
    if (n != secs[i].bytes) return invalid("bound file: section size differs from the header's counts");
    try {
      data[i].resize(std::max<size_t>(n, 4));
    } catch (const std::bad_alloc&) {
      set_error("host allocation for the bound file failed");
      return BBC_ENOMEM;
    }
    if ((e = read_exact(f, data[i].data(), n, h))) return e;
  }
  uint64_t hash = 0;
  Fnv dummy;
  if ((e = read_exact(f, &hash, 8, dummy))) return e;
  if (hash != h.h) return invalid("bound file checksum mismatch");
  if ((e = check_loaded(fh, data, secs, b))) return e;
  // The file is sound: only now touch the device.
  BBC_HIP(hipGetDevice(&b->device));
  for (size_t i = 0; i < secs.size(); ++i)
    if ((e = copy_in(*secs[i].buf, data[i].data(), secs[i].bytes, BBC_MEM_HOST, b, s))) return e;
  if ((e = launch_leaf_groups(b, nullptr, uint32_t(fh.n_leaves), s))) return e;
  BBC_HIP(hipStreamSynchronize(s));  // the host staging vectors go out of scope below
  DevScene& d = b->scene;
  d.n_tri = fh.n_tri;
  d.pos = static_cast<const float*>(b->pos.p);
  d.nrm = static_cast<const float*>(b->nrm.p);
  d.n_emit = fh.n_emit;
  d.epos = static_cast<const float*>(b->epos.p);
  d.eI = static_cast<const float*>(b->eI.p);
  d.eedge = fh.has_edges ? static_cast<const float*>(b->eedge.p) : nullptr;
  d.eta = fh.eta;
  for (int k = 0; k < 3; ++k) {
    d.q0[k] = fh.q0[k];
    d.f1[k] = fh.f1[k];
    d.f2[k] = fh.f2[k];
  }
  d.n_tri2 = fh.n_tri2;
  d.pos2 = rr ? static_cast<const float*>(b->pos2.p) : nullptr;
  d.nrm2 = rr ? static_cast<const float*>(b->nrm2.p) : nullptr;
  d.tid = rr ? static_cast<const uint32_t*>(b->tid.p) : nullptr;
  b->host = fh.host;
  b->max_cell = fh.max_cell;
  return BBC_OK;
}


}  // namespace bbc

using namespace bbc;

extern "C" {

const char* bbc_last_error(void) { return g_err.c_str(); }

bbc_status bbc_rebuild_bounds(bbc_bounds* h, const bbc_scene* scene, const bbc_emitters* emitters,
                              const bbc_subdiv_params* params, void* stream) {
  if (!h) return invalid("null bounds handle");
  bbc_status e = validate(scene, emitters, params);
  if (e) return e;
  Bounds* b = reinterpret_cast<Bounds*>(h);
  int dev = 0;
  BBC_HIP(hipGetDevice(&dev));
  if (dev != b->device) return invalid("current device differs from the handle's device");
  const hipStream_t s = as_stream(stream);
  if ((e = load_scene(b, scene, emitters, params, s))) return e;
  return run_build(b, s);
}

bbc_status bbc_build_bounds(const bbc_scene* scene, const bbc_emitters* emitters, const bbc_subdiv_params* params,
                            void* stream, bbc_bounds** out) {
  if (!out) return invalid("null output handle pointer");
  *out = nullptr;
  bbc_status e = validate(scene, emitters, params);
  if (e) return e;
  Bounds* b = new (std::nothrow) Bounds();
  if (!b) {
    set_error("host allocation failed");
    return BBC_ENOMEM;
  }
  BBC_HIP(hipGetDevice(&b->device));
  const hipStream_t s = as_stream(stream);
  if ((e = load_scene(b, scene, emitters, params, s)) || (e = run_build(b, s))) {
    (void)hipStreamSynchronize(s);
    release_all(b);
    delete b;
    return e;
  }
  *out = reinterpret_cast<bbc_bounds*>(b);
  return BBC_OK;
}

bbc_status bbc_free_bounds(bbc_bounds* h) {
  if (!h) return BBC_OK;
  Bounds* b = reinterpret_cast<Bounds*>(h);
  (void)hipDeviceSynchronize();
  release_all(b);
  release_graph(b->qgraph);
  release_graph(b->bgraph);
  for (hipEvent_t ev : b->tev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : b->bev)
    if (ev) (void)hipEventDestroy(ev);
  delete b;
  return BBC_OK;
}

bbc_status bbc_bounds_save(const bbc_bounds* h, const char* path) {
  if (!h || !path) return invalid("null bounds handle or path");
  Bounds* b = const_cast<Bounds*>(reinterpret_cast<const Bounds*>(h));
  FileHeader fh{};
  std::memcpy(fh.magic, kFileMagic, 8);
  fh.version = kFileVersion;
  fh.header_bytes = sizeof(FileHeader);
  const DevScene& d = b->scene;
  fh.chain = d.chain;
  fh.has_edges = d.eedge != nullptr;
  fh.rec_floats = b->rec_floats;
  fh.eta = d.eta;
  fh.n_tri = d.n_tri;
  fh.n_tri2 = d.n_tri2;
  fh.n_emit = d.n_emit;
  fh.n_tuples = b->n_tuples;
  fh.n_dense = b->n_dense;
  fh.n_leaves = b->n_leaves;
  fh.n_entries = b->n_entries;
  fh.max_cell = b->max_cell;
  for (int k = 0; k < 3; ++k) {
    fh.q0[k] = d.q0[k];
    fh.f1[k] = d.f1[k];
    fh.f2[k] = d.f2[k];
  }
  fh.params = b->params;
  fh.host = b->host;
  const std::vector<Section> secs = bound_sections(b, d.n_tri, d.n_tri2, d.n_emit, d.eedge != nullptr);
  std::vector<char> buf;
  for (const Section& sec : secs) {
    if (sec.bytes > sec.buf->bytes) return invalid("bounds handle holds no completed build");
  }
  FILE* f = std::fopen(path, "wb");
  if (!f) return invalid("cannot open the bound file for writing");
  Fnv hsh;
  bool ok = std::fwrite(&fh, sizeof fh, 1, f) == 1;
  hsh.add(&fh, sizeof fh);
  for (size_t i = 0; ok && i < secs.size(); ++i) {
    const uint64_t n = secs[i].bytes;
    try {
      buf.resize(std::max<size_t>(n, 1));
    } catch (const std::bad_alloc&) {
      std::fclose(f);
      set_error("host allocation for the bound file failed");
      return BBC_ENOMEM;
    }
    if (n) {
      const hipError_t he = hipMemcpy(buf.data(), secs[i].buf->p, n, hipMemcpyDeviceToHost);
      if (he != hipSuccess) {
        std::fclose(f);
        return hip_fail(he, "hipMemcpy (bound file)");
      }
    }
    ok = std::fwrite(&n, 8, 1, f) == 1 && (n == 0 || std::fwrite(buf.data(), 1, n, f) == n);
    hsh.add(&n, 8);
    hsh.add(buf.data(), n);
  }
  ok = ok && std::fwrite(&hsh.h, 8, 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return invalid("writing the bound file failed");
  return BBC_OK;
}

bbc_status bbc_bounds_load(const char* path, void* stream, bbc_bounds** out) {
  if (!out) return invalid("null output handle pointer");
  *out = nullptr;
  if (!path) return invalid("null path");
  FILE* f = std::fopen(path, "rb");
  if (!f) return invalid("cannot open the bound file");
  Bounds* b = new (std::nothrow) Bounds();
  if (!b) {
    std::fclose(f);
    set_error("host allocation failed");
    return BBC_ENOMEM;
  }
  const bbc_status e = load_file(f, b, as_stream(stream));
  std::fclose(f);
  if (e) {
    if (b->device_bytes) (void)hipStreamSynchronize(as_stream(stream));
    release_all(b);
    delete b;
    return e;
  }
  *out = reinterpret_cast<bbc_bounds*>(b);
  return BBC_OK;
}

bbc_status bbc_bounds_info(const bbc_bounds* h, bbc_bounds_info_t* out) {
  if (!h || !out) return invalid("null argument");
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  out->n_tuples = b->n_dense;
  out->n_live_tuples = b->host.n_live;
  out->n_boxes = int64_t(b->host.n_boxes) + int64_t(b->host.n_fp64);
  out->n_leaves = b->n_leaves;
  out->n_grid_entries = b->n_entries;
  out->n_inf_leaves = b->host.n_inf;
  out->n_fp64_boxes = int64_t(b->host.n_fp64) + int64_t(b->host.n_l0_fp64);
  out->device_bytes = b->device_bytes;
  out->grid_res = b->params.grid_res;
  out->max_depth_reached = int32_t(b->host.max_depth);
  out->n_cover_tuples = b->host.n_cover;
  return BBC_OK;
}

bbc_status bbc_export_leaves(const bbc_bounds* h, uint32_t* tuple, uint32_t* code, float* box, float* ukbox, float* E) {
  if (!h) return invalid("null bounds handle");
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  const size_t n = size_t(b->n_leaves);
  std::vector<uint32_t> t(n), c(n);
  std::vector<float> u(4 * n), e(2 * n);
  if (n) {
    BBC_HIP(hipMemcpy(t.data(), b->st.p, n * 4, hipMemcpyDeviceToHost));
    BBC_HIP(hipMemcpy(c.data(), b->sc.p, n * 4, hipMemcpyDeviceToHost));
    BBC_HIP(hipMemcpy(u.data(), b->su.p, n * 16, hipMemcpyDeviceToHost));
    BBC_HIP(hipMemcpy(e.data(), b->se.p, n * 8, hipMemcpyDeviceToHost));
  }
  if (tuple) {
    std::memcpy(tuple, t.data(), n * 4);
    if (b->scene.chain == BBC_CHAIN_RR && n) {
      std::vector<uint32_t> tid(size_t(b->n_tuples));
      BBC_HIP(hipMemcpy(tid.data(), b->tid.p, tid.size() * 4, hipMemcpyDeviceToHost));
      for (size_t i = 0; i < n; ++i) tuple[i] = tid[t[i]];
    }
  }
  if (code) std::memcpy(code, c.data(), n * 4);
  if (ukbox) std::memcpy(ukbox, u.data(), n * 16);
  if (E) std::memcpy(E, e.data(), n * 8);
  if (box) {
    std::vector<float> root(4 * size_t(b->n_tuples));
    BBC_HIP(hipMemcpy(root.data(), b->root.p, root.size() * 4, hipMemcpyDeviceToHost));
    for (size_t i = 0; i < n; ++i) {
      const float* r = &root[4 * size_t(t[i])];
      const int depth = int(c[i] >> 28);
      const uint32_t iu = (c[i] >> kCodeBits) & ((1u << kCodeBits) - 1), iv = c[i] & ((1u << kCodeBits) - 1);
      const float sc = std::ldexp(1.f, -depth);
      const float fu = (r[1] - r[0]) * sc, fv = (r[3] - r[2]) * sc;
      box[4 * i + 0] = r[0] + float(iu) * fu;
      box[4 * i + 1] = r[0] + float(iu + 1) * fu;
      box[4 * i + 2] = r[2] + float(iv) * fv;
      box[4 * i + 3] = r[2] + float(iv + 1) * fv;
    }
  }
  return BBC_OK;
}

bbc_status bbc_export_tuples(const bbc_bounds* h, uint32_t* tuples, int64_t cap, int64_t* n) {
  if (!h || !n) return invalid("null bounds handle or count");
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  *n = b->n_tuples;
  if (!tuples || cap <= 0) return BBC_OK;
  const int64_t m = std::min<int64_t>(cap, b->n_tuples);
  if (b->scene.chain == BBC_CHAIN_RR) {
    if (m) BBC_HIP(hipMemcpy(tuples, b->tid.p, size_t(m) * 4, hipMemcpyDeviceToHost));
  } else {
    for (int64_t t = 0; t < m; ++t) tuples[t] = uint32_t(t);
  }
  return BBC_OK;
}

bbc_status bbc_export_grid(const bbc_bounds* h, uint32_t* offsets, uint32_t* tuple, float* Et) {
  if (!h) return invalid("null bounds handle");
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  const int64_t nc = int64_t(b->params.grid_res) * b->params.grid_res;
  if (offsets) BBC_HIP(hipMemcpy(offsets, b->coff.p, size_t(nc + 2) * 4, hipMemcpyDeviceToHost));
  if (tuple && b->n_entries) {
    BBC_HIP(hipMemcpy(tuple, b->gt.p, size_t(b->n_entries) * 4, hipMemcpyDeviceToHost));
    if (b->scene.chain == BBC_CHAIN_RR) {  // report pair numbers, ascending like the indices
      std::vector<uint32_t> tid(size_t(b->n_tuples));
      BBC_HIP(hipMemcpy(tid.data(), b->tid.p, tid.size() * 4, hipMemcpyDeviceToHost));
      for (int64_t i = 0; i < b->n_entries; ++i) tuple[i] = tid[tuple[i]];
    }
  }
  if (Et && b->n_entries) BBC_HIP(hipMemcpy(Et, b->ge.p, size_t(b->n_entries) * 4, hipMemcpyDeviceToHost));
  return BBC_OK;
}

bbc_status bbc_query_irradiance_ex(const bbc_bounds* h, const float* points_dev, int64_t n, int32_t spp,
                                   uint64_t seed, int64_t point_index_base, int32_t mode, float* out_E_dev,
                                   float* stats_dev, bbc_query_stats* stats_host, void* stream) {
  if (!h) return invalid("null bounds handle");
  if (n < 0 || n > (int64_t(1) << 31)) return invalid("n must be in [0, 2^31]");
  if (n > 0 && (!points_dev || !out_E_dev)) return invalid("null points or output");
  if (spp < 1) return invalid("spp must be >= 1");
  if (point_index_base < 0) return invalid("point_index_base must be >= 0");
  const int form = mode & 15;
  if ((form != BBC_QUERY_FUSED && form != BBC_QUERY_STAGED) ||
      (mode & ~(15 | BBC_QUERY_EXHAUSTIVE | BBC_QUERY_SAMPLERS)))
    return invalid("unknown query mode");
  if ((mode & BBC_QUERY_SAMPLERS) && (form != BBC_QUERY_STAGED || (mode & BBC_QUERY_EXHAUSTIVE)))
    return invalid("the uniform, one-sample and bin samplers need the staged form without EXHAUSTIVE");
  Bounds* b = const_cast<Bounds*>(reinterpret_cast<const Bounds*>(h));
  const hipStream_t s = as_stream(stream);
  bbc_status e;
  float* st = stats_dev;
  DevBuf tmp_stats;
  if (stats_host && !st && n > 0) {
    if ((e = ensure(tmp_stats, size_t(n) * 16, nullptr))) return e;
    st = static_cast<float*>(tmp_stats.p);
  }
  unsigned long long* ctr = nullptr;
  if (stats_host) {
    if ((e = ensure(b->qcounters, 64, b))) return e;
    ctr = static_cast<unsigned long long*>(b->qcounters.p);
    if ((e = launch_fill_u32(reinterpret_cast<uint32_t*>(ctr), 0u, 16, s))) return e;
  }
  if (form == BBC_QUERY_STAGED)
    e = launch_query_staged(b, points_dev, n, spp, seed, point_index_base, mode, out_E_dev, st, ctr, s);
  else
    e = launch_query(b, points_dev, n, spp, seed, point_index_base, mode, out_E_dev, st, ctr, s);
  if (e) {
    release(tmp_stats);
    return e;
  }
  if (stats_host) {
    std::memset(stats_host, 0, sizeof(*stats_host));
    stats_host->n_points = n;
    unsigned long long c[8] = {0};
    BBC_HIP(hipMemcpyAsync(c, ctr, 64, hipMemcpyDeviceToHost, s));
    BBC_HIP(hipStreamSynchronize(s));
    stats_host->n_pairs = int64_t(c[0]);
    stats_host->n_newton = int64_t(c[1]);
    stats_host->n_iter_fp32 = int64_t(c[2]);
    stats_host->n_iter_fp64 = int64_t(c[3]);
    stats_host->n_roots = int64_t(c[4]);
    if (n > 0) {
      std::vector<float> hs(size_t(n) * 4);
      BBC_HIP(hipMemcpyAsync(hs.data(), st, hs.size() * 4, hipMemcpyDeviceToHost, s));
      BBC_HIP(hipStreamSynchronize(s));
      for (int64_t i = 0; i < n; ++i) {
        stats_host->sum_U += int64_t(hs[4 * i]);
        stats_host->sum_S += int64_t(hs[4 * i + 1]);
        stats_host->sum_varbound += hs[4 * i + 3];
      }
    }
  }
  release(tmp_stats);
  return BBC_OK;
}

bbc_status bbc_set_tuning(bbc_bounds* h, int32_t knob, int64_t value) {
  if (!h) return invalid("null bounds handle");
  Bounds* b = reinterpret_cast<Bounds*>(h);
  switch (knob) {
    case BBC_TUNE_QUERY_WAVES:
      if (value != 2 && value != 4) return invalid("query waves must be 2 or 4");
      b->tune.query_waves = int(value);
      return BBC_OK;
    case BBC_TUNE_QUERY_GRID:
      if (value < 1 || value > (1 << 20)) return invalid("query grid must be in [1, 2^20]");
      b->tune.query_grid = int(value);
      return BBC_OK;
    case BBC_TUNE_BUILD_GRID_PER_CU:
      if (value < 0 || value > 64) return invalid("build grid per CU must be in [0, 64]");
      b->tune.build_grid_per_cu = int(value);
      return BBC_OK;
    case BBC_TUNE_QUERY_TILE:
      if (value != 16 && value != 32 && value != 64) return invalid("query tile must be 16, 32 or 64");
      b->tune.query_tile = int(value);
      return BBC_OK;
    case BBC_TUNE_TIMING:
      if (value != 0 && value != 1) return invalid("timing must be 0 or 1");
      if (value && !b->bev[0]) {
        BBC_HIP(hipEventCreate(&b->bev[0]));
        BBC_HIP(hipEventCreate(&b->bev[1]));
      }
      if (value && b->tev.empty()) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        BBC_HIP(hipEventCreate(&e0));
        b->tev.push_back(e0);
        BBC_HIP(hipEventCreate(&e1));
        b->tev.push_back(e1);
      }
      b->tune.timing = int(value);
      return BBC_OK;
    case BBC_TUNE_NEWTON_STEPS:
      if (value < 0 || value > 20) return invalid("Newton steps per pass must be in [0, 20]");
      b->tune.newton_steps = int(value);
      return BBC_OK;
    case BBC_TUNE_NEWTON_RESULTS:
      if (value < 1 || value > 96) return invalid("Newton result buffer must be in [1, 96]");
      b->tune.newton_results = int(value);
      return BBC_OK;
    case BBC_TUNE_STAGED_PAIRS:
      if (value < 1 || value > int64_t(kMaxStagedPairs)) return invalid("staged pairs must be in [1, 2^28]");
      b->tune.staged_pairs = value;
      return BBC_OK;
    case BBC_TUNE_GRAPH:
      if (value != 0 && value != 1) return invalid("graph must be 0 or 1");
      b->tune.graph = int(value);
      return BBC_OK;
    case BBC_TUNE_RR_OUTLINED:
      if (value != 0 && value != 1) return invalid("rr_outlined must be 0 or 1");
      b->tune.rr_outlined = int(value);
      return BBC_OK;
    case BBC_TUNE_NEWTON_GRID_PER_CU:
      if (value < 0 || value > 64) return invalid("newton grid per CU must be in [0, 64]");
      b->tune.newton_grid_per_cu = int(value);
      return BBC_OK;
    case BBC_TUNE_BUILD_GRAPH:
      if (value != 0 && value != 1) return invalid("build graph must be 0 or 1");
      b->tune.build_graph = int(value);
      return BBC_OK;
    case BBC_TUNE_SUBDIV_SPLIT:
      if (value < 0 || value > (int64_t(1) << 20)) return invalid("subdivision split must be in [0, 2^20]");
      b->tune.subdiv_split = int(value);
      b->srec_cap = 0;  // sized again by the next build
      return BBC_OK;
    default:
      return invalid("unknown tuning knob");
  }
}

bbc_status bbc_get_tuning(const bbc_bounds* h, int32_t knob, int64_t* value) {
  if (!h || !value) return invalid("null argument");
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  switch (knob) {
    case BBC_TUNE_QUERY_WAVES: *value = b->tune.query_waves; return BBC_OK;
    case BBC_TUNE_QUERY_GRID: *value = b->tune.query_grid; return BBC_OK;
    case BBC_TUNE_BUILD_GRID_PER_CU: *value = b->tune.build_grid_per_cu; return BBC_OK;
    case BBC_TUNE_QUERY_TILE: *value = b->tune.query_tile; return BBC_OK;
    case BBC_TUNE_TIMING: *value = b->tune.timing; return BBC_OK;
    case BBC_TUNE_NEWTON_STEPS: *value = b->tune.newton_steps; return BBC_OK;
    case BBC_TUNE_NEWTON_RESULTS: *value = b->tune.newton_results; return BBC_OK;
    case BBC_TUNE_STAGED_PAIRS: *value = b->tune.staged_pairs; return BBC_OK;
    case BBC_TUNE_GRAPH: *value = b->tune.graph; return BBC_OK;
    case BBC_TUNE_RR_OUTLINED: *value = b->tune.rr_outlined; return BBC_OK;
    case BBC_TUNE_NEWTON_GRID_PER_CU: *value = b->tune.newton_grid_per_cu; return BBC_OK;
    case BBC_TUNE_BUILD_GRAPH: *value = b->tune.build_graph; return BBC_OK;
    case BBC_TUNE_SUBDIV_SPLIT: *value = b->tune.subdiv_split; return BBC_OK;
    default: return invalid("unknown tuning knob");
  }
}

bbc_status bbc_query_kernel_ms(const bbc_bounds* h, float* ms) {
  if (!h || !ms) return invalid("null argument");
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  if (!b->tune.timing || b->tev_used == 0) return invalid("no timed query on this handle (enable BBC_TUNE_TIMING)");
  float sum = 0.f;
  for (int k = 0; k < b->tev_used; ++k) {
    float t = 0.f;
    BBC_HIP(hipEventSynchronize(b->tev[2 * k + 1]));
    BBC_HIP(hipEventElapsedTime(&t, b->tev[2 * k], b->tev[2 * k + 1]));
    sum += t;
  }
  *ms = sum;
  return BBC_OK;
}

bbc_status bbc_build_kernel_ms(const bbc_bounds* h, float* ms, int32_t* launches) {
  if (!h || !ms) return invalid("null argument");
  const Bounds* b = reinterpret_cast<const Bounds*>(h);
  if (!b->tune.timing || !b->bev_recorded) return invalid("no timed build on this handle (enable BBC_TUNE_TIMING)");
  BBC_HIP(hipEventSynchronize(b->bev[1]));
  BBC_HIP(hipEventElapsedTime(ms, b->bev[0], b->bev[1]));
  if (launches) *launches = b->subdiv_launches;
  return BBC_OK;
}

bbc_status bbc_query_irradiance(const bbc_bounds* b, const float* points_dev, int64_t n, int32_t spp, uint64_t seed,
                                float* out_E_dev, bbc_query_stats* stats_host, void* stream) {
  return bbc_query_irradiance_ex(b, points_dev, n, spp, seed, 0, BBC_QUERY_FUSED, out_E_dev, nullptr, stats_host,
                                 stream);
}

}  // extern "C"
