// Host side of libptafs: data-set preparation, workspace management, the
// evaluation pipeline and the HMC driver (with HIP-graph trajectories).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "common.h"
#include "pool.h"

constexpr int kDefaultTilesPerChunk = 16;

// Device memory of a data set comes from a library-owned stream-ordered pool
// (one per device) and goes back to it with hipFreeAsync: neither allocation
// nor release synchronises the device, so data sets created and destroyed on
// their own streams do not stall the work of other streams.  Every call
// orders itself after the data set's previous work (an event recorded at the
// end of each call) and host waits are on that event only.
struct ptafs_dataset {
  int device = 0;
  pt::Dev base{};
  std::vector<int64_t> off;
  std::vector<void *> allocs;
  size_t ds_bytes = 0;
  hipMemPool_t pool = nullptr;
  hipStream_t aux = nullptr;          // library stream of the device (tuning changes, release)
  hipEvent_t done = nullptr;          // recorded after the data set's last enqueued work
  // tuning and chunk table of the TOA pass
  int tiles_per_chunk = kDefaultTilesPerChunk, wpb = 1, xcd_map = 1;
  bool chunks_dirty = true;
  int32_t *d_chunk = nullptr;
  std::vector<int32_t> chunk_host;    // source of the last chunk-table upload
  std::vector<int> psr_nchunks;
  // offset in the chunk table of the balanced placement for n_cb chain
  // blocks (index n_cb <= kMaxMapCb), or -1
  std::vector<int> wgmap_off;
  int n_chunks = 0;
  // workspace
  void *ws = nullptr;
  size_t ws_bytes = 0;
  // HMC scratch
  void *hmc = nullptr;
  size_t hmc_bytes = 0;
  // cached trajectory graph
  hipGraphExec_t gexec = nullptr;
  hipGraph_t graph = nullptr;
  hipStream_t cap = nullptr;          // private stream used only for graph capture
  struct GraphKey {
    int n_chains, n_leapfrog;
    double eps;
    const void *inv_mass, *x, *logp, *grad, *acc, *samples, *invalid;
    uint64_t seed;
    int tiles, wpb, xcd;
    void *ws, *hmc;
    bool operator==(const GraphKey &o) const { return std::memcmp(this, &o, sizeof(*this)) == 0; }
  } gkey{};
};

namespace {

#define PT_TRY(expr)                                  \
  do {                                                \
    hipError_t e_ = (expr);                           \
    if (e_ != hipSuccess) return PTAFS_E_HIP;         \
  } while (0)

#define PT_RC(expr)                                   \
  do {                                                \
    const int r_ = (expr);                            \
    if (r_) return r_;                                \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// One pool and one library stream per device, created on first use and kept
// until the process ends.  Freed blocks stay in the pool (no release
// threshold), so the next data set reuses them without a runtime allocation.
struct DevRes {
  hipMemPool_t pool = nullptr;
  hipStream_t aux = nullptr;
};
std::mutex g_res_mu;
std::map<int, DevRes> g_res;

int device_res(int dev, DevRes *out) {
  std::lock_guard<std::mutex> lk(g_res_mu);
  auto it = g_res.find(dev);
  if (it != g_res.end()) {
    *out = it->second;
    return PTAFS_OK;
  }
  DevRes r;
  hipMemPoolProps props{};
  props.allocType = hipMemAllocationTypePinned;
  props.handleTypes = hipMemHandleTypeNone;
  props.location.type = hipMemLocationTypeDevice;
  props.location.id = dev;
  PT_TRY(hipMemPoolCreate(&r.pool, &props));
  uint64_t keep = UINT64_MAX;
  PT_TRY(hipMemPoolSetAttribute(r.pool, hipMemPoolAttrReleaseThreshold, &keep));
  PT_TRY(hipStreamCreateWithFlags(&r.aux, hipStreamNonBlocking));
  g_res[dev] = r;
  *out = r;
  return PTAFS_OK;
}

int dalloc(ptafs_dataset *ds, void **p, size_t bytes, hipStream_t s) {
  *p = nullptr;
  if (hipMallocFromPoolAsync(p, std::max<size_t>(bytes, 8), ds->pool, s) != hipSuccess) {
    *p = nullptr;
    return PTAFS_E_NOMEM;
  }
  return PTAFS_OK;
}

void dfree(void *p, hipStream_t s) {
  if (p) (void)hipFreeAsync(p, s);
}

// Order a call on stream s after the data set's previous work (which may have
// been enqueued on another stream); mark the end of a call.
int begin_call(ptafs_dataset *ds, hipStream_t s) {
  PT_TRY(hipStreamWaitEvent(s, ds->done, 0));
  return PTAFS_OK;
}
int end_call(ptafs_dataset *ds, hipStream_t s) {
  PT_TRY(hipEventRecord(ds->done, s));
  return PTAFS_OK;
}


struct WsLayout {
  size_t coef_rn, coef_dm, lstore, sqk_rn, sqk_dm, cwc, part_rn, part_dm, part_chi, part_cw,
      bar_rn, bar_dm, chi_p, cw_p, dth_k, drn_k, ddm_k, flag_k, flag_dense, flag_out, st_pre, total;
};

WsLayout ws_layout(const pt::Dev &B, int c_pad, int n_chunks) {
  WsLayout L{};
  const size_t n = B.n_psr, cp = c_pad, ncb = c_pad / 16, nwg = (size_t)n_chunks * ncb;
  const size_t kmax = std::max(B.ka, B.nf_dm);
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align256(std::max<size_t>(bytes, 8));
    return r;
  };
  const size_t D8 = sizeof(double);
  L.coef_rn = take(n * B.rows_rn * cp * D8);
  L.coef_dm = take(n * B.rows_dm * cp * D8);
  L.lstore = take(cp * B.nf_gw * pt::chol_store_doubles(B.n_psr) * D8);
  L.sqk_rn = take(cp * B.ka * B.n_psr * D8);
  L.sqk_dm = take(cp * B.nf_dm * B.n_psr * D8);
  L.cwc = take(B.has_cw ? n * pt::kCwConst * cp * D8 : 0);
  L.part_rn = take(nwg * B.rows_rn * 16 * D8);
  L.part_dm = take(nwg * B.rows_dm * 16 * D8);
  L.part_chi = take(nwg * 16 * D8);
  L.part_cw = take(nwg * 8 * 16 * D8);
  L.bar_rn = take(n * B.rows_rn * cp * D8);
  L.bar_dm = take(n * B.rows_dm * cp * D8);
  L.chi_p = take(n * cp * D8);
  L.cw_p = take(n * 8 * cp * D8);
  L.dth_k = take(cp * B.ka * 2 * D8);
  L.drn_k = take(cp * B.ka * n * 2 * D8);
  L.ddm_k = take(cp * B.nf_dm * n * 2 * D8);
  L.flag_k = take(cp * kmax * sizeof(int32_t));
  L.flag_dense = take(cp * B.nf_gw * sizeof(int32_t));
  L.flag_out = take(cp * (kmax + pt::kSpecSeg) * sizeof(int32_t));
  L.st_pre = take(cp * sizeof(int32_t));
  L.total = o;
  return L;
}

int cpad_of(int n_chains) { return ((n_chains + 15) / 16) * 16; }

constexpr int kMaxMapCb = 16;   // chain blocks (256 chains) up to which placements are built

// Balanced placement of the TOA pass's work items on the compute units.  When
// the whole grid is resident at once, workgroup b runs on XCD b % n_xcd and
// shares its compute unit with b + n_cu, b + 2 n_cu, ... (the dispatcher's
// order, measured), and a compute unit's time is set by the TOAs of the
// chunks it holds.  The chunks go into bundles of k = workgroups per compute
// unit with near-equal TOA sums (largest first, each to the lightest bundle
// with room); a bundle's chain blocks take n_cb compute units of one XCD, one
// chain block each, so that every compute unit holds one bundle and the n_cb
// workgroups that read a chunk's TOAs share an L2.  The result only moves
// work between workgroups: each work item, and the order in which its
// partials are reduced, is the same under any placement.  Returns false when
// the grid does not have this shape.
bool balanced_map(const std::vector<int32_t> &cbg, const std::vector<int32_t> &cen, int n_cb, int n_cu,
                  int n_xcd, std::vector<int32_t> &map) {
  const int nc = (int)cbg.size();
  const long G = (long)nc * n_cb;
  if (nc == 0 || n_cb < 1 || n_cu <= 0 || n_xcd <= 0 || n_cu % n_xcd || G % n_cu) return false;
  const int k = (int)(G / n_cu), m = n_cu / n_xcd;   // workgroups per CU, CUs per XCD
  if (k < 1 || k > 8 || m % n_cb) return false;
  const int nb = n_cu / n_cb;                         // bundles, k chunks each
  if ((long)nb * k != nc) return false;
  std::vector<int> ord(nc);
  for (int c = 0; c < nc; ++c) ord[c] = c;
  std::stable_sort(ord.begin(), ord.end(),
                   [&](int a, int b) { return cen[a] - cbg[a] > cen[b] - cbg[b]; });
  std::vector<long> load(nb, 0);
  std::vector<int> cnt(nb, 0), memb((size_t)nb * k);
  for (int c : ord) {
    int best = -1;
    for (int b = 0; b < nb; ++b)
      if (cnt[b] < k && (best < 0 || load[b] < load[best])) best = b;
    memb[(size_t)best * k + cnt[best]++] = c;
    load[best] += cen[c] - cbg[c];
  }
  // then swap a chunk of the heaviest bundle with a lighter one of another
  // bundle (lightest bundles first) while that lowers the heaviest load
  auto sz = [&](int c) { return (long)(cen[c] - cbg[c]); };
  std::vector<int> by_load(nb);
  for (int it = 0; it < 4 * nc; ++it) {
    const int hb = (int)(std::max_element(load.begin(), load.end()) - load.begin());
    for (int b = 0; b < nb; ++b) by_load[b] = b;
    std::stable_sort(by_load.begin(), by_load.end(), [&](int a, int b) { return load[a] < load[b]; });
    bool moved = false;
    for (int ob : by_load) {
      if (ob == hb) continue;
      for (int i = 0; i < k && !moved; ++i)
        for (int j = 0; j < k && !moved; ++j) {
          int &a = memb[(size_t)hb * k + i], &b = memb[(size_t)ob * k + j];
          const long d = sz(a) - sz(b);
          if (d > 0 && std::max(load[hb] - d, load[ob] + d) < load[hb]) {
            std::swap(a, b);
            load[hb] -= d;
            load[ob] += d;
            moved = true;
          }
        }
      if (moved) break;
    }
    if (!moved) break;
  }
  map.assign((size_t)G, -1);
  for (int b = 0; b < nb; ++b) {
    const int x = b % n_xcd, r = b / n_xcd;
    for (int i = 0; i < k; ++i)
      for (int j = 0; j < n_cb; ++j) {
        const long w = (long)i * n_cu + (long)(r * n_cb + j) * n_xcd + x;
        map[(size_t)w] = memb[(size_t)b * k + i] * n_cb + j;
      }
  }
  std::vector<char> seen((size_t)G, 0);   // a permutation of the work items
  for (int32_t v : map) {
    if (v < 0 || v >= G || seen[(size_t)v]) return false;
    seen[(size_t)v] = 1;
  }
  return true;
}

// Split every pulsar into chunks of about `tpc` 16-TOA tiles (tile-aligned),
// then append the balanced placements of the chain-block counts whose grid
// has their shape.
void build_chunks(ptafs_dataset *ds, std::vector<int32_t> &tab) {
  const int n = ds->base.n_psr;
  const int tpc = std::max(1, ds->tiles_per_chunk);
  std::vector<int32_t> cps, cbg, cen;
  std::vector<int32_t> first(n + 1, 0);
  ds->psr_nchunks.assign(n, 0);
  for (int p = 0; p < n; ++p) {
    const int64_t b = ds->off[p], e = ds->off[p + 1];
    const int64_t tiles = (e - b + 15) / 16;
    const int64_t nch = std::max<int64_t>(1, (tiles + tpc - 1) / tpc);
    first[p] = (int32_t)cps.size();
    for (int64_t i = 0; i < nch; ++i) {
      const int64_t t0 = (i * tiles) / nch, t1 = ((i + 1) * tiles) / nch;
      cps.push_back(p);
      cbg.push_back((int32_t)(b + 16 * t0));
      cen.push_back((int32_t)std::min<int64_t>(e, b + 16 * t1));
    }
    ds->psr_nchunks[p] = (int)nch;
  }
  first[n] = (int32_t)cps.size();
  ds->n_chunks = (int)cps.size();
  tab.clear();
  tab.insert(tab.end(), cps.begin(), cps.end());
  tab.insert(tab.end(), cbg.begin(), cbg.end());
  tab.insert(tab.end(), cen.begin(), cen.end());
  tab.insert(tab.end(), first.begin(), first.end());
  ds->wgmap_off.assign(kMaxMapCb + 1, -1);
  std::vector<int32_t> map;
  for (int ncb = 1; ncb <= kMaxMapCb; ++ncb)
    if (balanced_map(cbg, cen, ncb, ds->base.n_cu, ds->base.n_xcd, map)) {
      ds->wgmap_off[ncb] = (int)tab.size();
      tab.insert(tab.end(), map.begin(), map.end());
    }
}

// A captured trajectory graph holds the addresses of the chunk table, the
// workspace and the HMC buffer in its kernel arguments: it is dropped whenever
// one of them is released.  The host first waits for the data set's own last
// work (the graph may still be running), never for the whole device.
int drop_graph(ptafs_dataset *ds) {
  if (!ds->gexec && !ds->graph) return PTAFS_OK;
  PT_TRY(hipEventSynchronize(ds->done));
  if (ds->gexec) (void)hipGraphExecDestroy(ds->gexec);
  if (ds->graph) (void)hipGraphDestroy(ds->graph);
  ds->gexec = nullptr;
  ds->graph = nullptr;
  return PTAFS_OK;
}

// (Re)build the chunk table on stream s, ordered after the data set's
// previous work; the old table goes back to the pool in stream order.
int ensure_chunks(ptafs_dataset *ds, hipStream_t s) {
  if (!ds->chunks_dirty) return PTAFS_OK;
  int rc = drop_graph(ds);
  if (rc) return rc;
  // the host table of the previous upload may still be read by that copy
  PT_TRY(hipEventSynchronize(ds->done));
  build_chunks(ds, ds->chunk_host);
  const std::vector<int32_t> &tab = ds->chunk_host;
  PT_RC(begin_call(ds, s));
  dfree(ds->d_chunk, s);
  ds->d_chunk = nullptr;
  void *p = nullptr;
  rc = dalloc(ds, &p, tab.size() * sizeof(int32_t), s);
  if (rc) return rc;
  ds->d_chunk = static_cast<int32_t *>(p);
  PT_TRY(hipMemcpyAsync(ds->d_chunk, tab.data(), tab.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  PT_RC(end_call(ds, s));
  const int nc = ds->n_chunks;
  ds->base.n_chunks = nc;
  ds->base.tiles_per_chunk = ds->tiles_per_chunk;
  ds->base.chunk_psr = ds->d_chunk;
  ds->base.chunk_begin = ds->d_chunk + nc;
  ds->base.chunk_end = ds->d_chunk + 2 * nc;
  ds->base.psr_chunk0 = ds->d_chunk + 3 * nc;
  ds->chunks_dirty = false;
  return PTAFS_OK;
}

// Grow the workspace on stream s (after begin_call on s).
int ensure_ws(ptafs_dataset *ds, int n_chains, hipStream_t s) {
  const WsLayout L = ws_layout(ds->base, cpad_of(n_chains), ds->n_chunks);
  if (L.total <= ds->ws_bytes) return PTAFS_OK;
  int rc = drop_graph(ds);
  if (rc) return rc;
  dfree(ds->ws, s);
  ds->ws = nullptr;
  ds->ws_bytes = 0;
  rc = dalloc(ds, &ds->ws, L.total, s);
  if (rc) return rc;
  PT_TRY(hipMemsetAsync(ds->ws, 0, L.total, s));   // every region starts at zero
  ds->ws_bytes = L.total;
  return PTAFS_OK;
}

pt::Dev make_dev(const ptafs_dataset *ds, int n_chains, void *ws) {
  pt::Dev D = ds->base;
  D.n_chains = n_chains;
  D.c_pad = cpad_of(n_chains);
  D.n_cb = D.c_pad / 16;
  D.wg_map = nullptr;
  if (ds->xcd_map == 2 && D.n_cb <= kMaxMapCb && (int)ds->wgmap_off.size() > D.n_cb &&
      ds->wgmap_off[D.n_cb] >= 0)
    D.wg_map = ds->d_chunk + ds->wgmap_off[D.n_cb];
  const WsLayout L = ws_layout(ds->base, D.c_pad, ds->n_chunks);
  char *w = static_cast<char *>(ws);
  D.coef_rn = reinterpret_cast<double *>(w + L.coef_rn);
  D.coef_dm = reinterpret_cast<double *>(w + L.coef_dm);
  D.lstore = reinterpret_cast<double *>(w + L.lstore);
  D.sqk_rn = reinterpret_cast<double *>(w + L.sqk_rn);
  D.sqk_dm = reinterpret_cast<double *>(w + L.sqk_dm);
  D.cwc = reinterpret_cast<double *>(w + L.cwc);
  D.part_rn = reinterpret_cast<double *>(w + L.part_rn);
  D.part_dm = reinterpret_cast<double *>(w + L.part_dm);
  D.part_chi = reinterpret_cast<double *>(w + L.part_chi);
  D.part_cw = reinterpret_cast<double *>(w + L.part_cw);
  D.bar_rn = reinterpret_cast<double *>(w + L.bar_rn);
  D.bar_dm = reinterpret_cast<double *>(w + L.bar_dm);
  D.chi_p = reinterpret_cast<double *>(w + L.chi_p);
  D.cw_p = reinterpret_cast<double *>(w + L.cw_p);
  D.dth_k = reinterpret_cast<double *>(w + L.dth_k);
  D.drn_k = reinterpret_cast<double *>(w + L.drn_k);
  D.ddm_k = reinterpret_cast<double *>(w + L.ddm_k);
  D.flag_k = reinterpret_cast<int32_t *>(w + L.flag_k);
  D.flag_dense = reinterpret_cast<int32_t *>(w + L.flag_dense);
  D.flag_out = reinterpret_cast<int32_t *>(w + L.flag_out);
  D.st_pre = reinterpret_cast<int32_t *>(w + L.st_pre);
  return D;
}

std::once_flag g_lds_once;
hipError_t g_lds_err = hipSuccess;

void set_lds_limits() {
  const size_t plain = (size_t)2 * (64 + 64) * 64 * sizeof(double);
  g_lds_err = ptk::set_plain_lds_limit(plain);
}

int enqueue_eval(ptafs_dataset *ds, int C, const double *x, double *logp, double *grad,
                 int32_t *status, hipStream_t s, bool plain, const pt::Kick *kick = nullptr,
                 void *ws = nullptr) {
  const pt::Dev D = make_dev(ds, C, ws ? ws : ds->ws);
  PT_TRY(ptk::launch_spectral_fwd(D, x, s));
  if (plain) {
    for (int p = 0; p < D.n_psr; ++p) PT_TRY(ptk::launch_toa_plain_psr(D, p, ds->psr_nchunks[p], s));
  } else {
    PT_TRY(ptk::launch_toa_mfma(D, ds->wpb, ds->xcd_map, s));
  }
  PT_TRY(ptk::launch_reduce_chunks(D, s));
  PT_TRY(ptk::launch_spectral_bwd(D, x, grad, s));
  PT_TRY(ptk::launch_finalize(D, x, logp, grad, status, s, kick));
  return PTAFS_OK;
}

int eval(ptafs_dataset *ds, int C, const double *x, double *logp, double *grad, int32_t *status,
         void *stream, bool plain) {
  if (!ds || C < 0) return PTAFS_E_ARG;
  if (C == 0) return PTAFS_OK;
  if (!x || !logp || !grad || !status) return PTAFS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  PT_TRY(hipSetDevice(ds->device));
  int rc = ensure_chunks(ds, s);
  if (rc) return rc;
  PT_RC(begin_call(ds, s));
  rc = ensure_ws(ds, C, s);
  if (rc) return rc;
  rc = enqueue_eval(ds, C, x, logp, grad, status, s, plain);
  if (rc) return rc;
  return end_call(ds, s);
}

template <typename T>
int upload(ptafs_dataset *ds, const T *src, size_t count, const T **dst, hipStream_t s) {
  void *p = nullptr;
  const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
  const int rc = dalloc(ds, &p, bytes, s);
  if (rc) return rc;
  ds->allocs.push_back(p);
  ds->ds_bytes += bytes;
  if (count) PT_TRY(hipMemcpyAsync(p, src, count * sizeof(T), hipMemcpyHostToDevice, s));
  *dst = static_cast<const T *>(p);
  return PTAFS_OK;
}

// Release everything a data set holds: wait for its own last work, then hand
// the blocks back to the pool on the library stream (no device-wide wait).
void free_all(ptafs_dataset *ds) {
  if (!ds) return;
  (void)hipSetDevice(ds->device);
  if (ds->done) (void)hipEventSynchronize(ds->done);
  if (ds->gexec) (void)hipGraphExecDestroy(ds->gexec);
  if (ds->graph) (void)hipGraphDestroy(ds->graph);
  if (ds->cap) (void)hipStreamDestroy(ds->cap);
  if (ds->aux) {
    for (void *p : ds->allocs) dfree(p, ds->aux);
    dfree(ds->d_chunk, ds->aux);
    dfree(ds->ws, ds->aux);
    dfree(ds->hmc, ds->aux);
  }
  if (ds->done) (void)hipEventDestroy(ds->done);
  delete ds;
}

// Validate a descriptor and fill the sizes and offsets of a device view
// (no device pointers, no GPU calls).
int plan(const ptafs_dataset_desc *d, pt::Dev &B) {
  B = pt::Dev{};
  if (!d) return PTAFS_E_ARG;
  const int n = d->n_psr;
  if (n < 1 || !d->toa_offsets) return PTAFS_E_ARG;
  if (n > PTAFS_MAX_PSR) return PTAFS_E_LIMIT;
  if (d->nf_rn < 0 || d->nf_gw < 0 || d->nf_dm < 0) return PTAFS_E_ARG;
  const int ka = std::max(d->nf_rn, d->nf_gw);
  const int kb = std::max(ka, d->nf_dm);
  if (kb > PTAFS_MAX_HARM) return PTAFS_E_LIMIT;
  if (!(d->tspan > 0.0) || d->n_backend < 1 || !d->efac || !d->equad || !d->psr_pos) return PTAFS_E_ARG;
  if (d->toa_offsets[0] != 0) return PTAFS_E_ARG;
  for (int p = 0; p < n; ++p)
    if (d->toa_offsets[p + 1] <= d->toa_offsets[p]) return PTAFS_E_ARG;
  const int64_t ntoa = d->toa_offsets[n];
  if (ntoa > (int64_t)INT32_MAX - 1024) return PTAFS_E_LIMIT;
  if (!d->t || !d->dt || !d->sigma || !d->nu || !d->backend) return PTAFS_E_ARG;
  for (int64_t i = 0; i < ntoa; ++i) {
    if (d->backend[i] < 0 || d->backend[i] >= d->n_backend) return PTAFS_E_ARG;
    if (!(d->sigma[i] > 0.0) || !(d->nu[i] > 0.0) || !std::isfinite(d->t[i]) || !std::isfinite(d->dt[i]))
      return PTAFS_E_ARG;
  }

  B.n_psr = n;
  B.n_toa = (int)ntoa;
  B.n_backend = d->n_backend;
  B.nf_rn = d->nf_rn;
  B.nf_gw = d->nf_gw;
  B.nf_dm = d->nf_dm;
  B.has_cw = d->has_cw ? 1 : 0;
  B.ka = ka;
  B.kb = kb;
  B.jt_rn = pt::tiles_for_pairs(kb + 2);
  B.jt_dm = d->nf_dm > 0 ? pt::tiles_for_pairs(d->nf_dm) : 0;
  B.rows_rn = 16 * B.jt_rn;
  B.rows_dm = 16 * B.jt_dm;
  B.n_free_rn = B.n_free_dm = 0;
  for (int r = 0; r < B.rows_rn; ++r) {
    const pt::Slot sl = pt::rn_slot(r, kb);
    if (sl.kind != 0 || sl.harm > ka) B.free_rn[B.n_free_rn++] = (int16_t)r;
  }
  for (int r = 0; r < B.rows_dm; ++r)
    if (pt::dm_slot(r, d->nf_dm).kind != 0) B.free_dm[B.n_free_dm++] = (int16_t)r;
  int o = 0;
  B.off_gw = o; o += d->nf_gw > 0 ? 2 : 0;
  B.off_rn = o; o += d->nf_rn > 0 ? 2 * n : 0;
  B.off_dm = o; o += d->nf_dm > 0 ? 2 * n : 0;
  B.off_cw = o; o += B.has_cw ? 8 : 0;
  B.n_theta = o;
  B.off_u = o; o += 3 * n;
  B.off_z = o; o += n * 2 * ka;
  B.off_zdm = o; o += n * 2 * d->nf_dm;
  B.d = o;
  B.tspan = d->tspan;
  B.dm_scale = d->dm_scale;
  B.sigma_b = d->sigma_b;
  if (B.n_theta > 0 && (!d->prior_lo || !d->prior_hi)) return PTAFS_E_ARG;
  double pc = 0.0;
  for (int i = 0; i < B.n_theta; ++i) {
    if (!(d->prior_hi[i] > d->prior_lo[i])) return PTAFS_E_ARG;
    pc -= std::log(d->prior_hi[i] - d->prior_lo[i]);
  }
  B.prior_const = pc;
  double tmax = 0.0;
  for (int64_t i = 0; i < ntoa; ++i) tmax = std::max(tmax, d->t[i]);
  B.tmax = tmax;
  return PTAFS_OK;
}

// Number of TOA chunks for a tiles-per-chunk setting (as build_chunks).
int count_chunks(const int64_t *off, int n, int tpc) {
  int64_t nc = 0;
  for (int p = 0; p < n; ++p) {
    const int64_t tiles = (off[p + 1] - off[p] + 15) / 16;
    nc += std::max<int64_t>(1, (tiles + tpc - 1) / tpc);
  }
  return (int)nc;
}

// Device bytes held by a data set (the uploads of ptafs_dataset_create and
// the chunk table).
size_t dataset_bytes_of(const pt::Dev &B, int n_chunks) {
  const size_t n = B.n_psr, ntoa = B.n_toa, npad = ntoa + pt::kToaPad;
  auto a = [](size_t count, size_t size) { return std::max<size_t>(count, 1) * size; };
  const int nt = pt::chol_tiles(B.n_psr);
  const size_t ntile = (size_t)(nt * (nt + 1) / 2) * 256;
  const size_t tiles = nt <= pt::kTileFwdMaxNT ? ntile : 0;
  size_t b = 7 * a(npad, 8) + 2 * a(ntoa, 8) + a(ntoa, 4) + 2 * a(B.n_backend, 8) + a(n + 1, 8) +
             2 * a(n, 8) + a(3 * n, 8) + a(n * n, 8) + a(n * (n + 1) / 2, 8) + 2 * a(tiles, 8) +
             2 * a(B.n_theta, 8) + a(PTAFS_MAX_HARM, 8);
  b += (size_t)(3 * n_chunks + n + 1) * sizeof(int32_t);
  return b;
}

// Scratch of ptafs_hmc_run for n_chains.
size_t hmc_bytes_of(const pt::Dev &B, int n_chains) {
  const size_t cd = (size_t)n_chains * B.d;
  return align256(3 * cd * sizeof(double)) +
         align256((1 + pt::kHmcBeginG) * (size_t)n_chains * sizeof(double)) +
         align256((size_t)n_chains * sizeof(int32_t)) + 256;
}

// Workspace of ptafs_logp_grad_noalloc: one array per device, part of the
// code object's data (each device that loads the library holds it until the
// process ends).  Host code never uses the symbol itself as an address: its
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

int scratch_ptr(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return PTAFS_E_LIMIT;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    PT_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));   // the current device is dev
    if (!p) return PTAFS_E_HIP;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PTAFS_OK;
}

}  // namespace

namespace ptr {
int device_pool(int dev, hipMemPool_t *pool, hipStream_t *aux) {
  DevRes r;
  const int rc = device_res(dev, &r);
  if (rc) return rc;
  *pool = r.pool;
  *aux = r.aux;
  return PTAFS_OK;
}
}  // namespace ptr

extern "C" {

int ptafs_logp_grad_noalloc(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                            double *grad, int32_t *status, void *stream) {
  if (!ds || n_chains < 0) return PTAFS_E_ARG;
  if (n_chains == 0) return PTAFS_OK;
  if (!x || !logp || !grad || !status) return PTAFS_E_ARG;
  // the chunk table is built by ptafs_dataset_create and ptafs_set_tuning;
  // rebuilding it here would allocate
  if (ds->chunks_dirty) return PTAFS_E_ARG;
  const WsLayout L = ws_layout(ds->base, cpad_of(n_chains), ds->n_chunks);
  if (L.total > kScratchBytes) return PTAFS_E_LIMIT;
  hipStream_t s = (hipStream_t)stream;
  PT_TRY(hipSetDevice(ds->device));
  void *ws = nullptr;
  PT_RC(scratch_ptr(ds->device, &ws));
  PT_RC(begin_call(ds, s));
  PT_RC(enqueue_eval(ds, n_chains, x, logp, grad, status, s, false, nullptr, ws));
  return end_call(ds, s);
}


const char *ptafs_strerror(int code) {
  switch (code) {
    case PTAFS_OK: return "success";
    case PTAFS_E_ARG: return "invalid argument or unsupported shape";
    case PTAFS_E_HIP: return "HIP runtime call failed";
    case PTAFS_E_NOMEM: return "device allocation failed";
    case PTAFS_E_LIMIT: return "size exceeds an implementation limit";
  }
  return "unknown error";
}

int ptafs_dataset_create(const ptafs_dataset_desc *d, void *stream, ptafs_dataset **out) {
  if (!d || !out) return PTAFS_E_ARG;
  *out = nullptr;
  pt::Dev plan_view;
  const int prc = plan(d, plan_view);
  if (prc) return prc;
  const int n = d->n_psr;
  const int64_t ntoa = d->toa_offsets[n];
  ptafs_dataset *ds = new (std::nothrow) ptafs_dataset();
  if (!ds) return PTAFS_E_NOMEM;
  if (hipGetDevice(&ds->device) != hipSuccess) {
    delete ds;
    return PTAFS_E_HIP;
  }
  std::call_once(g_lds_once, set_lds_limits);
  if (g_lds_err != hipSuccess) {
    delete ds;
    return PTAFS_E_HIP;
  }
  {
    DevRes res;
    const int r = device_res(ds->device, &res);
    if (r || hipEventCreateWithFlags(&ds->done, hipEventDisableTiming) != hipSuccess) {
      free_all(ds);
      return r ? r : PTAFS_E_HIP;
    }
    ds->pool = res.pool;
    ds->aux = res.aux;
  }
  hipStream_t s = (hipStream_t)stream;
  pt::Dev &B = ds->base;
  B = plan_view;
  if (hipDeviceGetAttribute(&B.n_cu, hipDeviceAttributeMultiprocessorCount, ds->device) != hipSuccess) {
    free_all(ds);
    return PTAFS_E_HIP;
  }
  // the XCD count only shapes the balanced placement: without it none is built
  if (hipDeviceGetAttribute(&B.n_xcd, hipDeviceAttributeNumberOfXccs, ds->device) != hipSuccess) {
    (void)hipGetLastError();
    B.n_xcd = 0;
  }
  // per-pulsar timing-model centring and the Hellings-Downs matrix
  std::vector<double> tc(n), tsi(n), gam((size_t)n * n);
  for (int p = 0; p < n; ++p) {
    double lo = d->t[d->toa_offsets[p]], hi = lo;
    for (int64_t i = d->toa_offsets[p]; i < d->toa_offsets[p + 1]; ++i) {
      lo = std::min(lo, d->t[i]);
      hi = std::max(hi, d->t[i]);
    }
    tc[p] = 0.5 * (lo + hi);
    const double hs = 0.5 * (hi - lo);
    tsi[p] = 1.0 / (hs > 0.0 ? hs : 1.0);
  }
  for (int I = 0; I < n; ++I)
    for (int J = 0; J < n; ++J) {
      if (I == J) {
        gam[(size_t)I * n + J] = 1.0;
        continue;
      }
      const double *a = d->psr_pos + 3 * I, *b = d->psr_pos + 3 * J;
      const double beta = 0.5 * (1.0 - (a[0] * b[0] + a[1] * b[1] + a[2] * b[2]));
      const double blb = beta > 0.0 ? beta * std::log(beta) : 0.0;
      gam[(size_t)I * n + J] = 1.5 * blb - 0.25 * beta + 0.5;
    }
  // chol(Gamma) for the adjoint of the common-process amplitude
  std::vector<double> gch((size_t)n * (n + 1) / 2, 0.0);
  {
    std::vector<double> Lf((size_t)n * n, 0.0);
    for (int j = 0; j < n; ++j) {
      double piv = gam[(size_t)j * n + j];
      for (int m = 0; m < j; ++m) piv -= Lf[(size_t)j * n + m] * Lf[(size_t)j * n + m];
      if (!(piv > 0.0)) {
        free_all(ds);
        return PTAFS_E_ARG;      // Gamma must be positive definite
      }
      const double ljj = std::sqrt(piv);
      Lf[(size_t)j * n + j] = ljj;
      for (int i = j + 1; i < n; ++i) {
        double t = gam[(size_t)i * n + j];
        for (int m = 0; m < j; ++m) t -= Lf[(size_t)i * n + m] * Lf[(size_t)j * n + m];
        Lf[(size_t)i * n + j] = t / ljj;
      }
    }
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) gch[(size_t)i * (i + 1) / 2 + j] = Lf[(size_t)i * n + j];
  }
  ds->off.assign(d->toa_offsets, d->toa_offsets + n + 1);
  // per-TOA basis phases, zero-padded for the prefetch of the TOA pass
  const size_t npad = (size_t)ntoa + pt::kToaPad;
  std::vector<double> vs(npad, 0.0), vc(npad, 0.0), vt(npad, 0.0), vw(npad, 0.0), vdt(npad, 0.0),
      vtt(npad, 0.0), vin(npad, 0.0);
  double lnn = 0.0;
  for (int p = 0; p < n; ++p)
    for (int64_t i = d->toa_offsets[p]; i < d->toa_offsets[p + 1]; ++i) {
      const double ph = pt::kTwoPi * (d->t[i] / d->tspan);
      vs[i] = std::sin(ph);
      vc[i] = std::cos(ph);
      vt[i] = (d->t[i] - tc[p]) * tsi[p];
      vw[i] = d->dm_scale / (d->nu[i] * d->nu[i]);
      vdt[i] = d->dt[i];
      vtt[i] = d->t[i];
      const int be = d->backend[i];
      const double es = d->efac[be] * d->sigma[i], eq = d->equad[be];
      const double N = es * es + eq * eq;
      vin[i] = 1.0 / N;
      lnn += std::log(N);
    }

  // host sources of the asynchronous uploads: alive until the stream is synchronised
  std::vector<double> gt, ht, lf;
  int rc = PTAFS_OK;
  auto chk = [&](int r) { if (r && !rc) rc = r; };
  chk(upload(ds, vtt.data(), npad, &B.t, s));
  chk(upload(ds, vdt.data(), npad, &B.dt, s));
  chk(upload(ds, vs.data(), npad, &B.sth, s));
  chk(upload(ds, vc.data(), npad, &B.cth, s));
  chk(upload(ds, vt.data(), npad, &B.tau, s));
  chk(upload(ds, vw.data(), npad, &B.wdm, s));
  chk(upload(ds, vin.data(), npad, &B.invn, s));
  B.lnn_total = lnn;
  chk(upload(ds, d->sigma, ntoa, &B.sigma, s));
  chk(upload(ds, d->nu, ntoa, &B.nu, s));
  chk(upload(ds, d->backend, ntoa, &B.backend, s));
  chk(upload(ds, d->efac, d->n_backend, &B.efac, s));
  chk(upload(ds, d->equad, d->n_backend, &B.equad, s));
  chk(upload(ds, d->toa_offsets, (size_t)n + 1, &B.toa_off, s));
  chk(upload(ds, tc.data(), n, &B.tau_c, s));
  chk(upload(ds, tsi.data(), n, &B.tau_sinv, s));
  chk(upload(ds, d->psr_pos, (size_t)3 * n, &B.pos, s));
  chk(upload(ds, gam.data(), (size_t)n * n, &B.gamma, s));
  chk(upload(ds, gch.data(), gch.size(), &B.gchol, s));
  {
    // the same factor as 16x16 tiles (tile (K, J) at K (K + 1) / 2 + J, row-major
    // inside), for the matrix-core adjoint of small arrays
    const int nt = pt::chol_tiles(n);
    if (nt <= pt::kTileFwdMaxNT) {
      gt.assign((size_t)(nt * (nt + 1) / 2) * 256, 0.0);
      for (int K = 0; K < nt; ++K)
        for (int J = 0; J <= K; ++J)
          for (int rr = 0; rr < 16; ++rr)
            for (int cc = 0; cc < 16; ++cc) {
              const int r = 16 * K + rr, k = 16 * J + cc;
              if (r < n && k <= r) gt[(size_t)(K * (K + 1) / 2 + J) * 256 + rr * 16 + cc] = gch[pt::pk(r, k)];
            }
    }
    chk(upload(ds, gt.data(), gt.size(), &B.gtile, s));
    if (nt <= pt::kTileFwdMaxNT) {
      ht.assign((size_t)(nt * (nt + 1) / 2) * 256, 0.0);
      for (int K = 0; K < nt; ++K)
        for (int J = 0; J <= K; ++J)
          for (int rr = 0; rr < 16; ++rr)
            for (int cc = 0; cc < 16; ++cc) {
              const int r = 16 * K + rr, k = 16 * J + cc;
              // column-major tiles (the register image of the forward's layout)
              if (r < n && k < n) ht[(size_t)(K * (K + 1) / 2 + J) * 256 + cc * 16 + rr] = gam[(size_t)r * n + k];
            }
    }
    chk(upload(ds, ht.data(), ht.size(), &B.gam_tile, s));
  }
  {
    // power-law spectra at f_k = (k + 1) / T in logarithms
    lf.assign(PTAFS_MAX_HARM, 0.0);
    for (int k = 0; k < PTAFS_MAX_HARM; ++k) lf[k] = std::log((k + 1) / d->tspan * pt::kYear);
    chk(upload(ds, lf.data(), lf.size(), &B.lnfy, s));
    B.pl_c = 3.0 * std::log(pt::kYear) - std::log(12.0 * pt::kPi * pt::kPi) - std::log(d->tspan);
  }
  chk(upload(ds, d->prior_lo, B.n_theta, &B.prior_lo, s));
  chk(upload(ds, d->prior_hi, B.n_theta, &B.prior_hi, s));
  if (!rc) rc = end_call(ds, s);
  if (!rc) rc = ensure_chunks(ds, s);
  // the host arrays above are the sources of the copies: wait for this
  // stream (the data set's own work) before they go out of scope, also on
  // the error path (the blocks go back to the pool only after the copies)
  if (hipStreamSynchronize(s) != hipSuccess && !rc) rc = PTAFS_E_HIP;
  if (rc) {
    free_all(ds);
    return rc;
  }
  *out = ds;
  return PTAFS_OK;
}

void ptafs_dataset_destroy(ptafs_dataset *ds) { free_all(ds); }

namespace {
void fill_layout(const pt::Dev &B, int n_chains, int n_chunks, ptafs_layout_info *out) {
  out->d = B.d;
  out->n_theta = B.n_theta;
  out->off_gw = B.off_gw;
  out->off_rn = B.off_rn;
  out->off_dm = B.off_dm;
  out->off_cw = B.off_cw;
  out->off_u = B.off_u;
  out->off_z = B.off_z;
  out->off_zdm = B.off_zdm;
  out->n_psr = B.n_psr;
  out->n_toa = B.n_toa;
  out->k_coef = B.ka;
  out->k_dm = B.nf_dm;
  out->dataset_bytes = dataset_bytes_of(B, n_chunks);
  out->workspace_bytes = ws_layout(B, cpad_of(n_chains), n_chunks).total;
  out->hmc_bytes = hmc_bytes_of(B, n_chains);
}
}  // namespace

int ptafs_layout(const ptafs_dataset *ds, int32_t n_chains, ptafs_layout_info *out) {
  if (!ds || !out || n_chains < 0) return PTAFS_E_ARG;
  fill_layout(ds->base, n_chains, count_chunks(ds->off.data(), ds->base.n_psr, ds->tiles_per_chunk), out);
  return PTAFS_OK;
}

int ptafs_estimate(const ptafs_dataset_desc *desc, int32_t n_chains, ptafs_layout_info *out) {
  if (!desc || !out || n_chains < 0) return PTAFS_E_ARG;
  pt::Dev B;
  const int rc = plan(desc, B);
  if (rc) return rc;
  fill_layout(B, n_chains, count_chunks(desc->toa_offsets, B.n_psr, kDefaultTilesPerChunk), out);
  return PTAFS_OK;
}

int ptafs_reserve(ptafs_dataset *ds, int32_t n_chains) {
  if (!ds || n_chains < 0) return PTAFS_E_ARG;
  PT_TRY(hipSetDevice(ds->device));
  hipStream_t s = ds->aux;
  int rc = ensure_chunks(ds, s);
  if (rc) return rc;
  PT_RC(begin_call(ds, s));
  rc = ensure_ws(ds, n_chains, s);
  if (rc) return rc;
  return end_call(ds, s);
}

int ptafs_logp_grad(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                    double *grad, int32_t *status, void *stream) {
  return eval(ds, n_chains, x, logp, grad, status, stream, false);
}

int ptafs_logp_grad_plain(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                          double *grad, int32_t *status, void *stream) {
  return eval(ds, n_chains, x, logp, grad, status, stream, true);
}

int ptafs_set_tuning(ptafs_dataset *ds, int32_t tiles_per_chunk, int32_t waves_per_block,
                     int32_t xcd_map) {
  if (!ds || tiles_per_chunk < 1 || tiles_per_chunk > 4096) return PTAFS_E_ARG;
  if (waves_per_block != 1 && waves_per_block != 2 && waves_per_block != 4) return PTAFS_E_ARG;
  if (xcd_map < 0 || xcd_map > 2) return PTAFS_E_ARG;
  if (tiles_per_chunk != ds->tiles_per_chunk) ds->chunks_dirty = true;
  ds->tiles_per_chunk = tiles_per_chunk;
  ds->wpb = waves_per_block;
  ds->xcd_map = xcd_map;
  PT_TRY(hipSetDevice(ds->device));
  return ensure_chunks(ds, ds->aux);
}

int ptafs_get_tuning(const ptafs_dataset *ds, int32_t *tiles_per_chunk, int32_t *waves_per_block,
                     int32_t *xcd_map) {
  if (!ds) return PTAFS_E_ARG;
  if (tiles_per_chunk) *tiles_per_chunk = ds->tiles_per_chunk;
  if (waves_per_block) *waves_per_block = ds->wpb;
  if (xcd_map) *xcd_map = ds->xcd_map;
  return PTAFS_OK;
}

int ptafs_profile_stages(ptafs_dataset *ds, int32_t n_chains, const double *x, double *logp,
                         double *grad, int32_t *status, int32_t reps, int32_t plain,
                         double *ms_out, void *stream) {
  if (!ds || n_chains < 1 || reps < 1 || !ms_out || !x || !logp || !grad || !status) return PTAFS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  PT_TRY(hipSetDevice(ds->device));
  int rc = ensure_chunks(ds, s);
  if (rc) return rc;
  PT_RC(begin_call(ds, s));
  rc = ensure_ws(ds, n_chains, s);
  if (rc) return rc;
  const pt::Dev D = make_dev(ds, n_chains, ds->ws);
  constexpr int kStages = 5;
  hipEvent_t ev[kStages + 1];
  for (auto &e : ev) PT_TRY(hipEventCreate(&e));
  double acc[kStages] = {0, 0, 0, 0, 0};
  int err = PTAFS_OK;
  for (int r = 0; r < reps && !err; ++r) {
    auto step = [&](int i, hipError_t e) {
      if (e != hipSuccess && !err) err = PTAFS_E_HIP;
      (void)hipEventRecord(ev[i + 1], s);
    };
    (void)hipEventRecord(ev[0], s);
    {
      step(0, ptk::launch_spectral_fwd(D, x, s));
    }
    if (plain) {
      hipError_t e = hipSuccess;
      for (int p = 0; p < D.n_psr && e == hipSuccess; ++p)
        e = ptk::launch_toa_plain_psr(D, p, ds->psr_nchunks[p], s);
      step(1, e);
    } else {
      step(1, ptk::launch_toa_mfma(D, ds->wpb, ds->xcd_map, s));
    }
    step(2, ptk::launch_reduce_chunks(D, s));
    {
      step(3, ptk::launch_spectral_bwd(D, x, grad, s));
    }
    step(4, ptk::launch_finalize(D, x, logp, grad, status, s));
    if (hipEventSynchronize(ev[kStages]) != hipSuccess) err = PTAFS_E_HIP;
    for (int i = 0; i < kStages && !err; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i], ev[i + 1]) != hipSuccess) err = PTAFS_E_HIP;
      acc[i] += ms;
    }
  }
  for (auto &e : ev) (void)hipEventDestroy(e);
  for (int i = 0; i < kStages; ++i) ms_out[i] = acc[i] / reps;
  if (!err) err = end_call(ds, s);
  return err;
}

int ptafs_hmc_run(ptafs_dataset *ds, int32_t n_chains, int32_t n_traj, int32_t n_leapfrog,
                  double eps, const double *inv_mass, uint64_t seed, uint64_t traj0, double *x,
                  double *logp, double *grad, int64_t *n_accept, double *samples,
                  int64_t *n_invalid, int32_t use_graph, void *stream) {
  if (!ds || n_chains < 0 || n_traj < 0 || n_leapfrog < 1 || !(eps > 0.0)) return PTAFS_E_ARG;
  if (n_chains == 0 || n_traj == 0) return PTAFS_OK;
  if (!x || !logp || !grad || !n_accept) return PTAFS_E_ARG;
  hipStream_t s = (hipStream_t)stream;
  PT_TRY(hipSetDevice(ds->device));
  int rc = ensure_chunks(ds, s);
  if (rc) return rc;
  PT_RC(begin_call(ds, s));
  rc = ensure_ws(ds, n_chains, s);
  if (rc) return rc;
  const int d = ds->base.d;
  const size_t cd = (size_t)n_chains * d;
  // scratch: p, x0, g0 [C][d], lp0 [C], kinetic-energy partials [C][kHmcBeginG],
  // status [C], trajectory counter
  const size_t need = hmc_bytes_of(ds->base, n_chains);
  if (need > ds->hmc_bytes) {
    rc = drop_graph(ds);
    if (rc) return rc;
    dfree(ds->hmc, s);
    ds->hmc = nullptr;
    ds->hmc_bytes = 0;
    rc = dalloc(ds, &ds->hmc, need, s);
    if (rc) return rc;
    ds->hmc_bytes = need;
  }
  char *h = static_cast<char *>(ds->hmc);
  double *p = reinterpret_cast<double *>(h);
  double *x0 = p + cd;
  double *g0 = x0 + cd;
  char *h2 = h + align256(3 * cd * sizeof(double));
  double *lp0 = reinterpret_cast<double *>(h2);
  double *h0 = lp0 + n_chains;
  char *h3 = h2 + align256((1 + pt::kHmcBeginG) * (size_t)n_chains * sizeof(double));
  int32_t *st = reinterpret_cast<int32_t *>(h3);
  uint64_t *traj = reinterpret_cast<uint64_t *>(h3 + align256((size_t)n_chains * sizeof(int32_t)));

  // trajectory counter and first trajectory of this run, set on the stream
  // (no host memory to keep alive, no synchronisation)
  PT_TRY(ptk::launch_traj_set(traj, traj0, s));

  const pt::Dev D = make_dev(ds, n_chains, ds->ws);
  auto one_traj = [&](hipStream_t q) -> int {
    PT_TRY(ptk::launch_hmc_begin(D, d, eps, inv_mass, seed, traj, x, logp, grad, p, x0, lp0, g0, h0, q));
    // every evaluation but the last ends with the kick and drift of its chain
    const pt::Kick kick{eps, inv_mass, x, p, n_invalid};
    for (int l = 0; l < n_leapfrog; ++l) {
      int r = enqueue_eval(ds, n_chains, x, logp, grad, st, q, false,
                           l + 1 < n_leapfrog ? &kick : nullptr);
      if (r) return r;
    }
    PT_TRY(ptk::launch_hmc_end(n_chains, d, eps, inv_mass, seed, traj, x, logp, grad, p, x0, lp0,
                               g0, h0, n_accept, samples, st, n_invalid, q));
    PT_TRY(ptk::launch_traj_inc(traj, q));
    return PTAFS_OK;
  };

  if (!use_graph) {
    for (int j = 0; j < n_traj; ++j) {
      rc = one_traj(s);
      if (rc) return rc;
    }
    return end_call(ds, s);
  }
  ptafs_dataset::GraphKey key{};
  std::memset(&key, 0, sizeof(key));
  key.n_chains = n_chains;
  key.n_leapfrog = n_leapfrog;
  key.eps = eps;
  key.inv_mass = inv_mass;
  key.x = x;
  key.logp = logp;
  key.grad = grad;
  key.acc = n_accept;
  key.samples = samples;
  key.invalid = n_invalid;
  key.seed = seed;
  key.tiles = ds->tiles_per_chunk;
  key.wpb = ds->wpb;
  key.xcd = ds->xcd_map;
  key.ws = ds->ws;
  key.hmc = ds->hmc;
  if (!ds->gexec || !(key == ds->gkey)) {
    // the previous graph may still run on the stream of an earlier call:
    // drop_graph waits for the data set's last work before destroying it
    rc = drop_graph(ds);
    if (rc) return rc;
    // Capture on a private stream (the caller's may be the null stream, which
    // cannot be captured); the graph is then launched on the caller's stream.
    if (!ds->cap) PT_TRY(hipStreamCreateWithFlags(&ds->cap, hipStreamNonBlocking));
    PT_TRY(hipStreamBeginCapture(ds->cap, hipStreamCaptureModeRelaxed));
    rc = one_traj(ds->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(ds->cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    if (ec != hipSuccess) return PTAFS_E_HIP;
    if (hipGraphInstantiate(&ds->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      return PTAFS_E_HIP;
    }
    ds->graph = g;
    ds->gkey = key;
  }
  for (int j = 0; j < n_traj; ++j) PT_TRY(hipGraphLaunch(ds->gexec, s));
  return end_call(ds, s);
}

}  // extern "C"
