// Batched interior-point driver (Section IV, Alg. 2) on one GPU.
//
// The paper runs Alg. 2 on a root processor plus N ranks that each own a
// slice of the L+M diagonal blocks and exchange the Schur complement, the
// right-hand sides and the dual steps by MPI every iteration.  Here all
// blocks of all systems of a batch live in one HBM arena; every step of the
// iteration is one kernel launch over the whole batch, the root's sums are
// in-kernel accumulations, and the only host traffic per iteration is a few
// scalars per system for the stopping decision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <string>
#include <map>
#include <mutex>
#include <vector>

#include "internal.h"
#include "kernels.h"

// Device scratch of the allocation-free solve (see scratch_ptr below).
static constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) char scratch[kScratchBytes];

namespace psdp {

namespace {

// Device blocks released by finished solves are kept (a few per device) and
// handed to later solves of no larger size, so that batches of the same
// shape do not pay hipMalloc / hipFree each call.
struct DevCache {
  std::mutex mu;
  struct Blk { int dev; void* p; size_t bytes; };
  std::vector<Blk> blks;
};
static DevCache g_cache;
constexpr size_t kCacheBlocks = 6;

static void* dev_alloc(size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return nullptr;
  {
    std::lock_guard<std::mutex> lk(g_cache.mu);
    size_t best = SIZE_MAX;
    int bi = -1;
    for (size_t i = 0; i < g_cache.blks.size(); ++i) {
      const auto& b = g_cache.blks[i];
      if (b.dev == dev && b.bytes >= bytes && b.bytes <= 2 * bytes + (1 << 20) && b.bytes < best) {
        best = b.bytes;
        bi = (int)i;
      }
    }
    if (bi >= 0) {
      void* p = g_cache.blks[bi].p;
      g_cache.blks.erase(g_cache.blks.begin() + bi);
      return p;
    }
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    // drop the cached blocks of this device and try once more
    std::lock_guard<std::mutex> lk(g_cache.mu);
    for (size_t i = 0; i < g_cache.blks.size();) {
      if (g_cache.blks[i].dev == dev) {
        hipFree(g_cache.blks[i].p);
        g_cache.blks.erase(g_cache.blks.begin() + i);
      } else {
        ++i;
      }
    }
    (void)hipGetLastError();
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
  }
  return p;
}

static void dev_release(void* p, size_t bytes) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) { hipFree(p); return; }
  std::lock_guard<std::mutex> lk(g_cache.mu);
  g_cache.blks.push_back({dev, p, bytes});
  while (g_cache.blks.size() > kCacheBlocks) {
    hipFree(g_cache.blks.front().p);
    g_cache.blks.erase(g_cache.blks.begin());
  }
}

struct StepTab {
  std::vector<int> sys, pre, first, cnt, tot;
  void add_step() {
    first.push_back((int)sys.size());
    cnt.push_back(0);
    tot.push_back(0);
  }
  void add(int s, int count) {
    sys.push_back(s);
    pre.push_back(tot.back());
    cnt.back() += 1;
    tot.back() += count;
  }
};

// HIP-event timing of launch classes on the solver stream.
struct Prof {
  bool on = false;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> ev;
  size_t next = 0;
  size_t base = 0;   // events below base belong to captured graphs
  std::vector<std::array<size_t, 3>> pend;
  double* out = nullptr;
  size_t mark() {
    if (!on) return 0;
    if (next == ev.size()) {
      hipEvent_t e;
      hipEventCreate(&e);
      ev.push_back(e);
    }
    hipEventRecord(ev[next], st);
    return next++;
  }
  void add(int cls, size_t a, size_t b) {
    if (on) pend.push_back({(size_t)cls, a, b});
  }
  // continue with n never-recorded events (created now, outside any capture)
  void fresh(size_t n) {
    if (!on) return;
    for (size_t i = 0; i < n; ++i) {
      hipEvent_t e;
      hipEventCreate(&e);
      ev.push_back(e);
    }
    next = ev.size() - n;
  }
  // after a stream synchronisation: accumulate and recycle the events
  void harvest() {
    if (!on) return;
    for (const auto& p : pend) {
      float ms = 0.f;
      hipEventElapsedTime(&ms, ev[p[1]], ev[p[2]]);
      out[2 * p[0]] += ms;
      out[2 * p[0] + 1] += 1.0;
    }
    pend.clear();
    next = base;
  }
  ~Prof() {
    for (auto e : ev) hipEventDestroy(e);
  }
};

// Host images of the per-batch tables.  They are needed only while a batch
// is built; their capacity stays with the thread, so that repeated solves of
// one shape reuse it instead of faulting in fresh pages each call.
struct HostTables {
  std::vector<BlkDesc> blk, pblk, dblk;
  std::vector<HMPair> pairs;
  std::vector<int64_t> offA1;
  std::vector<HM2> q2;
  std::vector<KTerm> terms;
  std::vector<AsmTile> tiles, ptiles;   // grouped tiles (n > 11), whole pairs (n <= 11)
  std::vector<int> csr_hh, csr_hid, csr_mh, csr_hl, csr_hm;   // per-system sections
  std::vector<int> csr_hh_off, csr_hid_off, csr_mh_off, csr_hl_off;
  std::vector<int> gpinfo;
  std::vector<int64_t> gpoff;
  std::vector<int> pq2b;                  // per system [n][n]: basis index of (p, q)
  std::vector<int64_t> pq2b_off;
  void clear() {
    blk.clear(); pblk.clear(); dblk.clear(); pairs.clear(); offA1.clear(); q2.clear();
    terms.clear(); tiles.clear(); ptiles.clear();
    csr_hh.clear(); csr_hid.clear(); csr_mh.clear(); csr_hl.clear(); csr_hm.clear();
    csr_hh_off.clear(); csr_hid_off.clear(); csr_mh_off.clear(); csr_hl_off.clear();
    gpinfo.clear(); gpoff.clear(); pq2b.clear(); pq2b_off.clear();
  }
};

static HostTables& host_tables() {
  static thread_local HostTables t;
  t.clear();
  return t;
}

// Pinned host buffers released by finished solves are kept (a few, bounded
// in bytes) and handed to later requests of about their size: pinning and
// unpinning cost tens of microseconds each.
struct PinCache {
  std::mutex mu;
  std::vector<std::pair<void*, size_t>> bufs;
  size_t bytes = 0;
};
static PinCache g_pin;
constexpr size_t kPinBuffers = 16;
constexpr size_t kPinBytes = size_t(1) << 30;

static void* pin_alloc(size_t bytes) {
  bytes = std::max<size_t>(bytes, 256);
  {
    std::lock_guard<std::mutex> lk(g_pin.mu);
    int bi = -1;
    for (size_t i = 0; i < g_pin.bufs.size(); ++i) {
      const size_t b = g_pin.bufs[i].second;
      if (b >= bytes && b <= 2 * bytes + (64 << 10) && (bi < 0 || b < g_pin.bufs[bi].second))
        bi = (int)i;
    }
    if (bi >= 0) {
      void* p = g_pin.bufs[bi].first;
      g_pin.bytes -= g_pin.bufs[bi].second;
      g_pin.bufs.erase(g_pin.bufs.begin() + bi);
      return p;
    }
  }
  void* p = nullptr;
  if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

// p must come from pin_alloc(bytes) with the same bytes
static void pin_release(void* p, size_t bytes) {
  if (!p) return;
  bytes = std::max<size_t>(bytes, 256);
  std::lock_guard<std::mutex> lk(g_pin.mu);
  g_pin.bufs.push_back({p, bytes});
  g_pin.bytes += bytes;
  while (g_pin.bufs.size() > kPinBuffers || g_pin.bytes > kPinBytes) {
    hipHostFree(g_pin.bufs.front().first);
    g_pin.bytes -= g_pin.bufs.front().second;
    g_pin.bufs.erase(g_pin.bufs.begin());
  }
}

struct StreamPool {
  std::mutex mu;
  std::vector<std::pair<int, hipStream_t>> idle;
};
static StreamPool g_streams;
constexpr size_t kPoolStreams = 8;

// a stream of device dev from the pool, or a new one (default priority)
static hipStream_t pool_take(int dev) {
  {
    std::lock_guard<std::mutex> lk(g_streams.mu);
    for (size_t i = 0; i < g_streams.idle.size(); ++i)
      if (g_streams.idle[i].first == dev) {
        hipStream_t st = g_streams.idle[i].second;
        g_streams.idle.erase(g_streams.idle.begin() + i);
        return st;
      }
  }
  hipStream_t st = nullptr;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return nullptr;
  return st;
}

// back to the pool once idle (or destroyed)
static void pool_give(int dev, hipStream_t st) {
  const bool ok = hipStreamSynchronize(st) == hipSuccess;
  std::lock_guard<std::mutex> lk(g_streams.mu);
  if (ok && g_streams.idle.size() < kPoolStreams) g_streams.idle.push_back({dev, st});
  else hipStreamDestroy(st);
}

struct Batch {
  Prof prof;
  int S = 0, maxn = 0, nblk = 0, npblk = 0, ndblk = 0, npairs = 0, nq2 = 0, ntiles = 0;
  int totL0 = 0, totK = 0, maxP = 0;
  std::vector<psdp_sdp*> sd;
  std::vector<SysDesc> sys;
  int maxn_pair = 0, nptiles = 0;
  std::vector<int> ownP, ownK;
  StepTab pan, trs, upd, wide, mid;
  StepTab lft;   // left-looking factorisation, one step per tile column
  StepTab fus;   // right-looking steps with the panel solve folded in
  StepTab lah, lal;   // look-ahead steps: tiles of the next column, tiles right of it
  // super-panel look-ahead: after super-panel s, the update of the next
  // super-panel's columns (lw1) runs on the solver stream and the update of
  // everything right of them (lw2) on a side stream, beside the next
  // super-panel's steps; the solver stream waits for it before the next lw1
  StepTab lw1, lw2;
  bool look = false;
  hipStream_t side = nullptr;
  int side_dev = 0;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool side_pending = false;
  // grouped solves of the systems not solved in one workgroup: per group q,
  // the diagonal-block sweeps (one per system), the row tiles below the
  // group (forward) and the column tiles left of it (backward)
  StepTab gin, gap, gfu, gbu;   // G_q inverses (one step); per group q: G_q
                                // products, row tiles below, column tiles left
  int maxNG = 0;
  std::vector<int> small_ids;
  int* d_small = nullptr;
  int64_t totblk = 0, totvec = 0, totlam = 0, totdg = 0, totP = 0, totpre = 0, totgi = 0, totpb = 0;

  // device
  void* dtab = nullptr;
  double* arena = nullptr;
  SysDesc* d_sys = nullptr;
  BlkDesc *d_blk = nullptr, *d_pblk = nullptr, *d_dblk = nullptr;
  HMPair* d_pairs = nullptr;
  int64_t* d_offA1 = nullptr;
  HM2* d_q2 = nullptr;
  KTerm* d_terms = nullptr;
  AsmTile* d_tiles = nullptr;
  AsmTile* d_ptiles = nullptr;
  int *d_gpinfo = nullptr, *d_ownP = nullptr, *d_ownK = nullptr;
  int64_t* d_gpoff = nullptr;
  int *d_pan_sys = nullptr, *d_pan_pre = nullptr, *d_upd_sys = nullptr, *d_upd_pre = nullptr;
  int *d_trs_sys = nullptr, *d_trs_pre = nullptr, *d_wide_sys = nullptr, *d_wide_pre = nullptr;
  int *d_lft_sys = nullptr, *d_lft_pre = nullptr;
  int *d_mid_sys = nullptr, *d_mid_pre = nullptr;
  int *d_fus_sys = nullptr, *d_fus_pre = nullptr;
  int *d_lah_sys = nullptr, *d_lah_pre = nullptr, *d_lal_sys = nullptr, *d_lal_pre = nullptr;
  int *d_lw1_sys = nullptr, *d_lw1_pre = nullptr, *d_lw2_sys = nullptr, *d_lw2_pre = nullptr;
  int *d_gin_sys = nullptr, *d_gin_pre = nullptr, *d_gap_sys = nullptr, *d_gap_pre = nullptr;
  int *d_gfu_sys = nullptr, *d_gfu_pre = nullptr, *d_gbu_sys = nullptr, *d_gbu_pre = nullptr;
  int* d_flags = nullptr;
  double* d_shf = nullptr;   // per system: diagonal shift factor of the Schur factorisation
  double* d_sc = nullptr;
  double* d_red = nullptr;
  int* d_kout = nullptr;
  double* d_cert = nullptr;
  // arena arrays
  double *X, *Z, *Zi, *G, *S1, *T1, *W1, *dXh, *dZh, *Wc, *dXb, *dZb, *dX, *dZ, *Cf;
  double *y, *dyh, *dyb, *r, *z, *BX, *rv1, *rv2, *ylift, *vtmp;
  bool any_phase1 = false;
  bool use_graph = false;   // replay each iteration's launches from hipGraphs
  std::vector<char> use_pair, use_small;   // kernel paths per system
  std::vector<int> use_sw, use_ssw;
  bool f32 = false;   // precision form: reduced-precision Schur assembly + refinement
  int prec = PSDP_PREC_FP64;
  int ir_max = 0;
  bool shift_pass = false;  // the launches being issued factor some system with a shift
  int graph_launches = 0;   // hipGraphLaunch calls of this solve
  std::vector<char> asm64;   // per system: fell back to FP64 assembly (sticky)
  int maxK = 0;
  int nmax_small = 0;   // largest block order <= kSmallN in the batch (0: none)
  int nmin_big = 0;     // the general block kernels skip orders below this
  double *Lam, *Ldiag, *Linv, *Ginv, *Pm, *pre, *rscr, *PB;

  // pinned host mirrors of the per-iteration transfers (flags, scalars),
  // one cached block
  int* h_hf = nullptr;
  int* h_prev = nullptr;
  double* h_shf = nullptr;
  double* h_sc = nullptr;
  void* h_pin = nullptr;
  size_t h_pin_bytes = 0;

  size_t dtab_bytes = 0, arena_bytes = 0;
  // external device memory (the allocation-free solve): tables and arena
  // are carved from ext, host images live in ordinary host vectors, and
  // nothing is released here
  char* ext = nullptr;
  size_t ext_bytes = 0;
  std::vector<char> h_img;

  ~Batch() {
    if (side) pool_give(side_dev, side);
    if (ev_fork) hipEventDestroy(ev_fork);
    if (ev_join) hipEventDestroy(ev_join);
    if (ext) return;
    if (dtab) dev_release(dtab, dtab_bytes);
    if (arena) dev_release(arena, arena_bytes);
    pin_release(h_pin, h_pin_bytes);
  }
};

// places table v at offset off of the device table block (base) and of its
// host image (stage); the image goes up in one copy once every table is in
struct Stage {
  char* p;
  size_t cap;
};

template <class T>
static int upload(void* base, const Stage& stage, size_t& off, const std::vector<T>& v, T** dptr) {
  *dptr = (T*)((char*)base + off);
  const size_t bytes = v.size() * sizeof(T);
  if (off + bytes > stage.cap) return fail(PSDP_EINVAL, "table image overflow");
  if (bytes) std::memcpy(stage.p + off, v.data(), bytes);
  off += (bytes + 255) / 256 * 256;
  return PSDP_OK;
}

template <class T>
static size_t tabsize(const std::vector<T>& v) {
  return (v.size() * sizeof(T) + 255) / 256 * 256;
}

// Builds every per-batch table on the host and allocates the arena.
// Kernel paths per system: whole-pair assembly (n^2 <= 128 only) or grouped
// tiles; the whole solve in one workgroup (P <= kSmallP only) or by groups
// of kSG tiles.
struct Choice {
  std::vector<char> pair, small;
  std::vector<int> sw;   // Schur Cholesky panels per super-panel (0: left-looking, -2: the
                         // right-looking steps with the panel solve folded in)
  std::vector<int> ssw;  // panels per sub-panel inside a super-panel (= sw: none)
};

// the whole-pair assembly kernel serves systems whose basis order n has
// n^2 <= 128 (the discrete form's terms are n x n blocks of its 2n x 2n
// products, read at their offsets)
static bool pair_ok(const psdp_sdp* p) { return p->n * p->n <= 128; }

static Choice default_choice(psdp_sdp* const* sdps, int count) {
  Choice c;
  for (int s = 0; s < count; ++s) {
    c.pair.push_back(pair_ok(sdps[s]));
    c.small.push_back(sdps[s]->Kpad / kNB <= kSmallP);
    c.sw.push_back(kSW);
    c.ssw.push_back(kSW);
  }
  return c;
}

static int build_batch(Batch& B, psdp_sdp* const* sdps, int count, const Choice* ch = nullptr) {
  // B.ext / B.ext_bytes, when set by the caller, replace every device allocation
  HostTables& H = host_tables();
  Choice dflt;
  if (!ch) {
    dflt = default_choice(sdps, count);
    ch = &dflt;
  }
  B.look = !B.ext;   // (the allocation-free solve keeps one stream)
  B.use_pair = ch->pair;
  B.use_small = ch->small;
  B.use_sw = ch->sw;
  B.use_ssw = ch->ssw;
  B.S = count;
  B.sd.assign(sdps, sdps + count);
  // ---- per-system layout
  int64_t curblk = 0, curvec = 0, curlam = 0, curdg = 0, curP = 0, curpre = 0, curgi = 0, curpb = 0;
  std::vector<std::vector<int64_t>> a1(count), a2(count), ay(count);
  std::vector<size_t> q2beg(count + 1, 0);
  B.ownP.push_back(0);
  B.ownK.push_back(0);
  for (int s = 0; s < count; ++s) {
    psdp_sdp* p = sdps[s];
    const int n = p->bo;   // block order
    const int64_t nn = (int64_t)n * n;
    B.maxn = std::max(B.maxn, n);
    if (n <= kSmallN) B.nmax_small = std::max(B.nmax_small, n);
    else B.nmin_big = kSmallN + 1;
    SysDesc d{};
    d.n = n; d.L0 = p->L0; d.L = p->L; d.M = p->M; d.Nt = p->Nt; d.nb = p->nb;
    d.nbas = p->n;
    d.copies = n / p->n;
    d.K = (int)p->K; d.Kpad = (int)p->Kpad; d.P = d.Kpad / kNB; d.mode = 0;
    d.sw = ch->sw[s];
    d.ssw = ch->ssw[s] > 0 && d.sw > 0 && d.sw % ch->ssw[s] == 0 ? ch->ssw[s] : d.sw;
    d.blk0 = (int)H.blk.size();
    d.boff = curblk;
    for (int j = 0; j < p->nb; ++j) {
      BlkDesc b{s, j, n, 0, curblk + j * nn};
      H.blk.push_back(b);
      (j < p->L ? H.pblk : H.dblk).push_back(b);
    }
    curblk += p->nb * nn;
    d.voff = curvec; curvec += d.Kpad;
    d.loff = curlam; curlam += (int64_t)d.Kpad * d.Kpad;
    d.dgoff = curdg; curdg += (int64_t)d.P * kNB * kNB;
    d.pboff = -1;
    if (d.sw == -2) {   // two panel slots of P tiles
      d.pboff = curpb;
      curpb += 2 * (int64_t)d.P * kNB * kNB;
    }
    d.gioff = -1;
    if (!(ch->small[s] && d.P <= kSmallP)) {   // grouped solves
      d.gioff = curgi;
      curgi += (int64_t)((d.P + kSG - 1) / kSG) * 2 * kGS * kGS;
    }
    d.poff = curP; curP += p->L0 * nn;
    d.H = p->dHh; d.betaf = p->dbetaf; d.cdiag = p->dcdiag; d.scale = p->dscale; d.basis = p->dbasis;
    B.maxP = std::max(B.maxP, d.P);
    // active (m, h) pairs, in (m, h) order
    a1[s].assign((size_t)p->M * p->L0, -1);
    a2[s].assign((size_t)p->M * p->L0, -1);
    ay[s].assign((size_t)p->M * p->L0, -1);
    const int pair0 = (int)H.pairs.size();
    std::vector<std::vector<int>> by_h(p->L0);
    H.csr_mh_off.push_back((int)H.csr_mh.size());
    H.csr_hl_off.push_back((int)H.csr_hl.size());
    int cnt_hl = 0;
    for (int m = 0; m < p->M; ++m) {
      H.csr_mh.push_back(cnt_hl);
      for (int h = 0; h < p->L0; ++h) {
        if (!p->hmask[m * p->L0 + h]) continue;
        HMPair hp{s, m, h, n, curpre, curpre + nn};
        ay[s][m * p->L0 + h] = curpre;
        a2[s][m * p->L0 + h] = curpre + nn;
        a1[s][m * p->L0 + h] = curpre + 2 * nn;
        H.offA1.push_back(curpre + 2 * nn);
        curpre += 3 * nn;
        by_h[h].push_back((int)H.pairs.size());
        H.pairs.push_back(hp);
        H.csr_hl.push_back(h);
        ++cnt_hl;
      }
    }
    H.csr_mh.push_back(cnt_hl);
    H.csr_hh_off.push_back((int)H.csr_hh.size());
    H.csr_hid_off.push_back((int)H.csr_hid.size());
    int cnt = 0;
    for (int h = 0; h < p->L0; ++h) {
      H.csr_hh.push_back(cnt);
      for (int id : by_h[h]) {
        H.csr_hid.push_back(id);
        H.csr_hm.push_back(H.pairs[id].m);
      }
      cnt += (int)by_h[h].size();
    }
    H.csr_hh.push_back(cnt);
    d.npairs_hm = (int)H.pairs.size() - pair0;
    // Schur pre-products A3/A4 for h <= h2 on every block with both active
    q2beg[s] = H.q2.size();
    for (int m = 0; m < p->M; ++m) {
      for (int h = 0; h < p->L0; ++h) {
        if (!p->hmask[m * p->L0 + h]) continue;
        for (int h2 = h; h2 < p->L0; ++h2) {
          if (!p->hmask[m * p->L0 + h2]) continue;
          HM2 q{s, m, h, h2, n, 0, curpre, curpre + nn, a1[s][m * p->L0 + h2], a2[s][m * p->L0 + h2]};
          curpre += 2 * nn;
          H.q2.push_back(q);
        }
      }
    }
    // entry (p, q) of a block -> its basis index (-1 off the diagonal copies
    // of the discrete form's blocks)
    H.pq2b_off.push_back((int64_t)H.pq2b.size());
    H.pq2b.resize(H.pq2b.size() + (size_t)nn, -1);
    {
      int* t = H.pq2b.data() + H.pq2b_off.back();
      for (int c = 0; c < d.copies; ++c)
        for (int b = 0; b < p->Nt; ++b) {
          const int pp = c * p->n + p->basis.pairs[2 * b], qq = c * p->n + p->basis.pairs[2 * b + 1];
          t[pp * n + qq] = b;
          t[qq * n + pp] = b;
        }
    }
    // basis group pairs
    H.gpoff.push_back((int64_t)H.gpinfo.size());
    const BasisInfo& bi = p->basis;
    for (int g = 0; g < bi.ngp; ++g) {
      H.gpinfo.push_back(bi.gp_g1[g]);
      H.gpinfo.push_back(bi.gp_g2[g]);
      H.gpinfo.push_back(bi.gp_off[g]);
      H.gpinfo.push_back(bi.gp_size[g]);
    }
    q2beg[s + 1] = H.q2.size();
    B.sys.push_back(d);
    B.ownP.push_back(B.ownP.back() + p->L0);
    B.ownK.push_back(B.ownK.back() + (int)p->K);
    B.maxK = std::max(B.maxK, (int)p->K);
  }
  // every arena array starts on a 256-byte boundary (vector loads of 16 bytes
  // and more need at least 16)
  B.totblk = round_up(curblk, 32);
  B.totvec = round_up(curvec, 32);
  B.totlam = round_up(curlam, 32);
  B.totdg = round_up(curdg, 32);
  B.totP = round_up(curP, 32);
  B.totpre = round_up(curpre, 32);
  B.totgi = round_up(curgi, 32);
  B.totpb = round_up(curpb, 32);
  B.nblk = (int)H.blk.size();
  B.npblk = (int)H.pblk.size();
  B.ndblk = (int)H.dblk.size();
  B.npairs = (int)H.pairs.size();
  B.nq2 = (int)H.q2.size();
  B.totL0 = B.ownP.back();
  B.totK = B.ownK.back();

  // ---- arena
  const int nblkarr = 15, nvec = 10;
  // whole-pair assembly scratch: one n^2 x n^2 slot per workgroup of its grid
  int pn = 0;
  for (int s = 0; s < count; ++s)
    if (ch->pair[s] && pair_ok(sdps[s])) pn = std::max(pn, sdps[s]->n);
  // (only blocks of order 11 keep R in global scratch; smaller ones in LDS)
  const int64_t totrs = pn * pn > 112 ? (int64_t)kPairGrid * pn * pn * pn * pn : 0;
  const int64_t total = nblkarr * B.totblk + nvec * B.totvec + B.totlam + 2 * B.totdg + B.totgi + B.totpb + B.totP +
                        B.totpre + totrs;
  B.arena_bytes = (size_t)std::max<int64_t>(total, 1) * 8;
  if (B.ext) {
    if (B.arena_bytes > B.ext_bytes)
      return fail(PSDP_EINVAL, "the solve needs " + std::to_string(B.arena_bytes) +
                                   " bytes of device scratch for its arena alone; the allocation-free "
                                   "entry point has " + std::to_string(B.ext_bytes));
    B.arena = (double*)B.ext;
  } else if (!(B.arena = (double*)dev_alloc(B.arena_bytes))) {
    return fail(PSDP_ENOMEM, "device allocation of the solver arena failed (" +
                                 std::to_string(total * 8) + " bytes)");
  }
  double* a = B.arena;
  int64_t o = 0;
  double** blkarrs[nblkarr] = {&B.X, &B.Z, &B.Zi, &B.G, &B.S1, &B.T1, &B.W1, &B.dXh,
                               &B.dZh, &B.Wc, &B.dXb, &B.dZb, &B.dX, &B.dZ, &B.Cf};
  for (int i = 0; i < nblkarr; ++i) { *blkarrs[i] = a + o; o += B.totblk; }
  double** vecs[nvec] = {&B.y, &B.dyh, &B.dyb, &B.r, &B.z, &B.BX, &B.rv1, &B.rv2, &B.ylift, &B.vtmp};
  for (int i = 0; i < nvec; ++i) { *vecs[i] = a + o; o += B.totvec; }
  B.Lam = a + o; o += B.totlam;
  B.Ldiag = a + o; o += B.totdg;
  B.Linv = a + o; o += B.totdg;
  B.Ginv = a + o; o += B.totgi;
  B.PB = a + o; o += B.totpb;
  B.Pm = a + o; o += B.totP;
  B.pre = a + o; o += B.totpre;
  B.rscr = a + o; o += totrs;
  const int64_t preBase = B.pre - a, ziBase = B.Zi - a, xBase = B.X - a;
  for (auto& hp : H.pairs) { hp.offY += preBase; hp.offA2 += preBase; }
  for (auto& v : H.offA1) v += preBase;
  for (auto& q : H.q2) { q.offA3 += preBase; q.offA4 += preBase; q.srcA1 += preBase; q.srcA2 += preBase; }

  // ---- Schur k-lists and tiles
  std::vector<int64_t> a3, a4;
  for (int s = 0; s < count; ++s) {
    psdp_sdp* p = sdps[s];
    const int L0 = p->L0, L = p->L, M = p->M;
    const int64_t nn = (int64_t)p->bo * p->bo;
    const int64_t b0 = B.sys[s].boff;
    // a term tr(E T E' U) of the expansion; on the discrete form's blocks the
    // basis matrices sit on the two diagonal copies, so the term becomes the
    // four terms of the copy pairs (c1, c2): T's block (c1, c2) with U's
    // block (c2, c1), read at shifted offsets of the order-2n matrices
    const int nbs = p->n, bo = p->bo, ncp = bo / nbs;
    auto add_term = [&](int64_t oT, int64_t oU, double c, int tT, int tU) {
      for (int c1 = 0; c1 < ncp; ++c1)
        for (int c2 = 0; c2 < ncp; ++c2) {
          const int64_t sT = tT ? (int64_t)c2 * nbs * bo + c1 * nbs : (int64_t)c1 * nbs * bo + c2 * nbs;
          const int64_t sU = tU ? (int64_t)c1 * nbs * bo + c2 * nbs : (int64_t)c2 * nbs * bo + c1 * nbs;
          H.terms.push_back(KTerm{oT + sT, oU + sU, c, tT, tU});
        }
    };
    // index of the A3/A4 of (m, h, h2), from the system's own pre-products
    a3.assign((size_t)M * L0 * L0, -1);
    a4.assign((size_t)M * L0 * L0, -1);
    for (size_t i = q2beg[s]; i < q2beg[s + 1]; ++i) {
      const HM2& q = H.q2[i];
      a3[((size_t)q.m * L0 + q.h) * L0 + q.h2] = q.offA3;
      a4[((size_t)q.m * L0 + q.h) * L0 + q.h2] = q.offA4;
    }
    for (int h = 0; h < L0; ++h) {
      for (int h2 = h; h2 < L0; ++h2) {
        const int kbeg = (int)H.terms.size();
        for (int j = 0; j < L; ++j) {
          if (!p->bmask[h * L + j] || !p->bmask[h2 * L + j]) continue;
          const double c = p->betaf[h * L + j] * p->betaf[h2 * L + j];
          add_term(ziBase + b0 + j * nn, xBase + b0 + j * nn, c, 0, 0);
        }
        for (int m = 0; m < M; ++m) {
          if (!p->hmask[m * L0 + h] || !p->hmask[m * L0 + h2]) continue;
          const int64_t bm = b0 + (int64_t)(L + m) * nn;
          const int64_t A1h = a1[s][m * L0 + h] + preBase, A1h2 = a1[s][m * L0 + h2] + preBase;
          const int64_t A2h = a2[s][m * L0 + h] + preBase, A2h2 = a2[s][m * L0 + h2] + preBase;
          const int64_t A3 = a3[((size_t)m * L0 + h) * L0 + h2];
          const int64_t A4 = a4[((size_t)m * L0 + h) * L0 + h2];
          add_term(A1h2, A2h, 1.0, 0, 0);         // (Zi H'^T, X H^T)
          add_term(ziBase + bm, A3, 1.0, 0, 1);   // (Zi, H' X H^T)
          add_term(A4, xBase + bm, 1.0, 0, 0);    // (H Zi H'^T, X)
          add_term(A1h, A2h2, 1.0, 1, 1);         // (H Zi, H' X)
        }
        const int kcnt = (int)H.terms.size() - kbeg;
        if (kcnt == 0) continue;   // the block stays zero
        if (ch->pair[s] && pair_ok(p)) {
          H.ptiles.push_back(AsmTile{s, h, h2, -1, -1, kbeg, kcnt, 0});
          B.maxn_pair = std::max(B.maxn_pair, p->n);
          continue;
        }
        const int ngp = p->basis.ngp;
        for (int rg = 0; rg < ngp; ++rg)
          for (int cg = (h == h2 ? rg : 0); cg < ngp; ++cg)
            H.tiles.push_back(AsmTile{s, h, h2, rg, cg, kbeg, kcnt, 0});
      }
    }
  }
  B.ntiles = (int)H.tiles.size();
  B.nptiles = (int)H.ptiles.size();

  // ---- Cholesky step tables
  for (int s = 0; s < count; ++s)
    if (ch->small[s] && B.sys[s].P <= kSmallP) B.small_ids.push_back(s);
  for (int pstep = 0; pstep < B.maxP; ++pstep) {
    B.pan.add_step();
    B.trs.add_step();
    B.upd.add_step();
    B.wide.add_step();
    B.mid.add_step();
    B.lft.add_step();
    B.fus.add_step();
    B.lah.add_step();
    B.lal.add_step();
    B.lw1.add_step();
    B.lw2.add_step();

    // last column of the narrow update of step q (super-panel end; a
    // super-panel followed by fewer than sw panels absorbs them, since
    // their wide update would be one long, nearly empty launch)
    auto sp_end = [](int P, int q, int sw) {
      const int se = (q / sw) * sw + sw - 1;
      return P - 1 - se < sw ? P - 1 : se;
    };
    // last panel of the sub-panel of q (sub-panels split a super-panel in
    // runs of ssw panels; the narrow updates stay inside one).  ssw = sw
    // means none: a super-panel that absorbed a short tail stays whole
    auto sub_end = [&](int P, int q, int sw, int ssw) {
      return ssw >= sw ? sp_end(P, q, sw) : std::min(sp_end(P, q, sw), (q / ssw) * ssw + ssw - 1);
    };
    for (int s = 0; s < count; ++s) {
      const int P = B.sys[s].P;
      if (P <= pstep) continue;
      if (B.sys[s].sw == -2) {   // one launch per step: the first diagonal, then the updates
        if (pstep == 0) B.pan.add(s, 1);
        int nn = 0;
        for (int j = pstep + 1; j < P; ++j) nn += P - j;
        if (nn > 0) B.fus.add(s, nn);
        continue;
      }
      if (B.sys[s].sw == -3) {   // look-ahead: diagonal and panel solve of column 0, then one launch per step
        if (pstep == 0) {
          B.pan.add(s, 1);
          if (P > 1) B.trs.add(s, P - 1);
        }
        if (pstep <= P - 2) {
          B.lah.add(s, P - pstep - 1);
          int nn = 0;
          for (int j = pstep + 2; j < P; ++j) nn += P - j;
          if (nn > 0) B.lal.add(s, nn);
        }
        continue;
      }
      if (B.sys[s].sw == 0) {   // left-looking: the tiles of column pstep
        B.lft.add(s, pstep == 0 ? 1 : P - pstep);
        continue;
      }
      // after a narrow update of step pstep - 1 its workgroup of tile
      // (pstep, pstep) has already factored the diagonal tile
      const int sw = B.sys[s].sw, ssw = B.sys[s].ssw;
      if (pstep == 0 || sub_end(P, pstep - 1, sw, ssw) < pstep) B.pan.add(s, 1);
      const int T = P - pstep - 1;
      if (T > 0) B.trs.add(s, T);
      // narrow update: columns p+1 .. end of the sub-panel
      const int se = sp_end(P, pstep, sw), sse = sub_end(P, pstep, sw, ssw);
      int nn = 0;
      for (int j = pstep + 1; j <= sse; ++j) nn += P - j;
      if (nn > 0) B.upd.add(s, nn);
      // sub-panel update after a sub-panel's last panel: rows below it,
      // columns up to the super-panel's end, in 128 x 128 blocks
      if (pstep == sse && pstep < se) {
        const int nrb = (P - pstep) / 2, ncb = (se - pstep + 1) / 2;
        B.mid.add(s, ncb * nrb - ncb * (ncb - 1) / 2);
      }
      // wide update after the super-panel's last panel
      if (pstep == se && pstep % sw == sw - 1 && pstep < P - 1) {
        if (B.look && ssw == sw) {
          // look-ahead: the next super-panel's columns (every row below),
          // then the tiles right of it
          const int ne = sp_end(P, pstep + 1, sw);
          const int nrb = (P - pstep) / 2, ncb = (ne - pstep + 1) / 2;
          B.lw1.add(s, ncb * nrb - ncb * (ncb - 1) / 2);
          if (ne < P - 1) {
            const int nb2 = (P - ne) / 2;
            B.lw2.add(s, nb2 * (nb2 + 1) / 2);
          }
        } else {
          const int nb2 = (P - pstep - 1 + 1) / 2;
          B.wide.add(s, nb2 * (nb2 + 1) / 2);
        }
      }

    }
  }

  if (!B.lw2.sys.empty()) {   // the side stream of the super-panel look-ahead
    PSDP_HIP(hipGetDevice(&B.side_dev));
    if (!(B.side = pool_take(B.side_dev))) return fail(PSDP_EDEVICE, "stream creation failed");
    PSDP_HIP(hipEventCreateWithFlags(&B.ev_fork, hipEventDisableTiming));
    PSDP_HIP(hipEventCreateWithFlags(&B.ev_join, hipEventDisableTiming));
  }

  // ---- grouped solve tables
  auto tiled = [&](int s) { return !(ch->small[s] && B.sys[s].P <= kSmallP); };
  for (int s = 0; s < count; ++s)
    if (tiled(s)) B.maxNG = std::max(B.maxNG, (B.sys[s].P + kSG - 1) / kSG);
  // G_q by doubling: step l (block halves of m = 2^l tiles) has kSG m / 2
  // output tiles per group; the last step covers every tile of the group
  for (int m = 1; m <= kSG; m *= 2) {
    B.gin.add_step();
    for (int s = 0; s < count; ++s)
      if (tiled(s)) B.gin.add(s, (B.sys[s].P + kSG - 1) / kSG * (m < kSG ? kSG * m / 2 : kSG * kSG));
  }
  for (int q = 0; q < B.maxNG; ++q) {
    B.gap.add_step();
    B.gfu.add_step();
    B.gbu.add_step();
    for (int s = 0; s < count; ++s) {
      const int P = B.sys[s].P;
      if (!tiled(s) || P <= kSG * q) continue;
      B.gap.add(s, (std::min(P, kSG * (q + 1)) - kSG * q) * (kNB / 16));
      if (P > kSG * (q + 1)) B.gfu.add(s, (P - kSG * (q + 1)) * (kNB / 16));
      if (q > 0) B.gbu.add(s, kSG * q * (kNB / kBwdCW));
    }
  }

  // ---- device tables
  size_t tb = 0;
  tb += tabsize(B.sys) + tabsize(H.blk) + tabsize(H.pblk) + tabsize(H.dblk) + tabsize(H.pairs);
  tb += tabsize(H.offA1) + tabsize(H.q2) + tabsize(H.terms) + tabsize(H.tiles) + tabsize(H.gpinfo);
  tb += tabsize(H.ptiles);
  tb += tabsize(H.gpoff) + tabsize(B.ownP) + tabsize(B.ownK) + tabsize(H.csr_hh) + tabsize(H.csr_hid);
  tb += tabsize(H.csr_mh) + tabsize(H.csr_hl) + tabsize(H.csr_hm) + tabsize(H.pq2b);
  tb += tabsize(B.pan.sys) + tabsize(B.pan.pre) + tabsize(B.upd.sys) + tabsize(B.upd.pre);
  tb += tabsize(B.trs.sys) + tabsize(B.trs.pre) + tabsize(B.wide.sys) + tabsize(B.wide.pre);
  tb += tabsize(B.lft.sys) + tabsize(B.lft.pre);
  tb += tabsize(B.mid.sys) + tabsize(B.mid.pre);
  tb += tabsize(B.fus.sys) + tabsize(B.fus.pre);
  tb += tabsize(B.lah.sys) + tabsize(B.lah.pre) + tabsize(B.lal.sys) + tabsize(B.lal.pre);
  tb += tabsize(B.lw1.sys) + tabsize(B.lw1.pre) + tabsize(B.lw2.sys) + tabsize(B.lw2.pre);
  tb += tabsize(B.gin.sys) + tabsize(B.gin.pre) + tabsize(B.gap.sys) + tabsize(B.gap.pre);
  tb += tabsize(B.gfu.sys) + tabsize(B.gfu.pre) + tabsize(B.gbu.sys) + tabsize(B.gbu.pre);
  tb += tabsize(B.small_ids);
  tb += ((size_t)B.S * 4 + 255) / 256 * 256 + ((size_t)B.S * kNSC * 8 + 255) / 256 * 256;
  tb += ((size_t)B.S * 8 + 255) / 256 * 256;   // shift factors
  tb += ((size_t)B.nblk * 4 * 8 + 255) / 256 * 256 + ((size_t)B.nblk * 2 * 4 + 255) / 256 * 256;
  tb += ((size_t)B.nblk * 2 * 8 + 255) / 256 * 256 + 4096;
  B.dtab_bytes = tb;
  const size_t arena_end = (B.arena_bytes + 255) / 256 * 256;
  if (B.ext) {
    if (arena_end + tb > B.ext_bytes)
      return fail(PSDP_EINVAL, "the solve needs " + std::to_string(arena_end + tb) +
                                   " bytes of device scratch; the allocation-free entry point has " +
                                   std::to_string(B.ext_bytes));
    B.dtab = B.ext + arena_end;
  } else if (!(B.dtab = dev_alloc(tb))) {
    return fail(PSDP_ENOMEM, "device allocation of tables failed");
  }
  size_t off = 0;
  int rc = PSDP_OK;
  static thread_local std::vector<char> ext_stage;
  if (B.ext && ext_stage.size() < tb) ext_stage.resize(tb);
  Stage stage{B.ext ? ext_stage.data() : (char*)pin_alloc(tb), tb};
  if (!stage.p) return fail(PSDP_ENOMEM, "pinned staging buffer for the tables");
  struct StageGuard {
    Stage& s;
    bool ext;
    ~StageGuard() { if (!ext) pin_release(s.p, s.cap); }
  } stage_guard{stage, B.ext != nullptr};
  int* d_csr_hh; int* d_csr_hid; int* d_csr_mh; int* d_csr_hl; int* d_csr_hm; int* d_pq2b;
  // the per-system CSR pointers must be patched into SysDesc before upload
  {
    char* base = (char*)B.dtab;
    size_t o2 = tabsize(B.sys) + tabsize(H.blk) + tabsize(H.pblk) + tabsize(H.dblk) + tabsize(H.pairs) +
                tabsize(H.offA1) + tabsize(H.q2) + tabsize(H.terms) + tabsize(H.tiles) +
                tabsize(H.ptiles) + tabsize(H.gpinfo) + tabsize(H.gpoff) + tabsize(B.ownP) +
                tabsize(B.ownK);
    d_csr_hh = (int*)(base + o2); o2 += tabsize(H.csr_hh);
    d_csr_hid = (int*)(base + o2); o2 += tabsize(H.csr_hid);
    d_csr_mh = (int*)(base + o2); o2 += tabsize(H.csr_mh);
    d_csr_hl = (int*)(base + o2); o2 += tabsize(H.csr_hl);
    d_csr_hm = (int*)(base + o2); o2 += tabsize(H.csr_hm);
    d_pq2b = (int*)(base + o2);
    for (int s = 0; s < count; ++s) {
      B.sys[s].pq2b = d_pq2b + H.pq2b_off[s];
      B.sys[s].hm_by_h = d_csr_hh + H.csr_hh_off[s];
      B.sys[s].hm_ids = d_csr_hid + H.csr_hid_off[s];
      B.sys[s].hm_m = d_csr_hm + H.csr_hid_off[s];
      B.sys[s].h_by_m = d_csr_mh + H.csr_mh_off[s];
      B.sys[s].h_list = d_csr_hl + H.csr_hl_off[s];
    }
  }
  if ((rc = upload(B.dtab, stage, off, B.sys, &B.d_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.blk, &B.d_blk))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.pblk, &B.d_pblk))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.dblk, &B.d_dblk))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.pairs, &B.d_pairs))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.offA1, &B.d_offA1))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.q2, &B.d_q2))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.terms, &B.d_terms))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.tiles, &B.d_tiles))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.ptiles, &B.d_ptiles))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.gpinfo, &B.d_gpinfo))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.gpoff, &B.d_gpoff))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.ownP, &B.d_ownP))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.ownK, &B.d_ownK))) return rc;
  int* tmp;
  if ((rc = upload(B.dtab, stage, off, H.csr_hh, &tmp))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.csr_hid, &tmp))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.csr_mh, &tmp))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.csr_hl, &tmp))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.csr_hm, &tmp))) return rc;
  if ((rc = upload(B.dtab, stage, off, H.pq2b, &tmp))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.pan.sys, &B.d_pan_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.pan.pre, &B.d_pan_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.trs.sys, &B.d_trs_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.trs.pre, &B.d_trs_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.wide.sys, &B.d_wide_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.wide.pre, &B.d_wide_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.upd.sys, &B.d_upd_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.upd.pre, &B.d_upd_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lft.sys, &B.d_lft_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lft.pre, &B.d_lft_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.mid.sys, &B.d_mid_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.mid.pre, &B.d_mid_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.fus.sys, &B.d_fus_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.fus.pre, &B.d_fus_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lah.sys, &B.d_lah_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lah.pre, &B.d_lah_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lal.sys, &B.d_lal_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lal.pre, &B.d_lal_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lw1.sys, &B.d_lw1_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lw1.pre, &B.d_lw1_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lw2.sys, &B.d_lw2_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.lw2.pre, &B.d_lw2_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gin.sys, &B.d_gin_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gin.pre, &B.d_gin_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gap.sys, &B.d_gap_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gap.pre, &B.d_gap_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gfu.sys, &B.d_gfu_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gfu.pre, &B.d_gfu_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gbu.sys, &B.d_gbu_sys))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.gbu.pre, &B.d_gbu_pre))) return rc;
  if ((rc = upload(B.dtab, stage, off, B.small_ids, &B.d_small))) return rc;
  PSDP_HIP(hipMemcpy(B.dtab, stage.p, off, hipMemcpyHostToDevice));
  char* base = (char*)B.dtab;
  B.d_flags = (int*)(base + off); off += ((size_t)B.S * 4 + 255) / 256 * 256;
  B.d_sc = (double*)(base + off); off += ((size_t)B.S * kNSC * 8 + 255) / 256 * 256;
  B.d_shf = (double*)(base + off); off += ((size_t)B.S * 8 + 255) / 256 * 256;
  B.d_red = (double*)(base + off); off += ((size_t)B.nblk * 4 * 8 + 255) / 256 * 256;
  B.d_kout = (int*)(base + off); off += ((size_t)B.nblk * 2 * 4 + 255) / 256 * 256;   // X and Z ladders
  B.d_cert = (double*)(base + off); off += ((size_t)B.nblk * 2 * 8 + 255) / 256 * 256;
  const size_t hf_bytes = ((size_t)B.S * 4 + 255) / 256 * 256;
  const size_t shf_bytes = ((size_t)B.S * 8 + 255) / 256 * 256;
  B.h_pin_bytes = 2 * hf_bytes + shf_bytes + (size_t)B.S * kNSC * 8;
  if (B.ext) {
    B.h_img.resize(B.h_pin_bytes);
    B.h_pin = B.h_img.data();
  } else if (!(B.h_pin = pin_alloc(B.h_pin_bytes))) {
    return fail(PSDP_ENOMEM, "pinned host buffers");
  }
  B.h_hf = (int*)B.h_pin;
  B.h_prev = (int*)((char*)B.h_pin + hf_bytes);
  B.h_shf = (double*)((char*)B.h_pin + 2 * hf_bytes);
  B.h_sc = (double*)((char*)B.h_pin + 2 * hf_bytes + shf_bytes);
  return PSDP_OK;
}

// ---------------------------------------------------------------------------
// operator helpers
// ---------------------------------------------------------------------------

// general block product, blocks above kSmallN only (the small ones take the
// fused kernels)
static void gemm_big(Batch& B, hipStream_t st, const double* A, const double* Bm, double* C,
                     double alpha, const double* D, double beta, int bslot) {
  if (B.maxn > kSmallN)
    launch_gemm_blocks(st, B.nblk, B.d_blk, B.d_flags, B.d_sc, A, 0, Bm, 0, C, alpha, -1, D, beta,
                       bslot, B.nmin_big, gemm_tiles(B.maxn));
}

// W1 = sym(Z^-1 A X) on every block
static void op_sym_ZAX(Batch& B, hipStream_t st, const double* A) {
  const int nskip = B.nmax_small ? kSmallN : 0;
  if (B.nmax_small) launch_sym_ZAX_small(st, B.nblk, B.nmax_small, B.d_blk, B.d_flags, B.Zi, A, B.X, B.W1);
  if (B.maxn > kSmallN) {
    gemm_big(B, st, B.Zi, A, B.T1, 1.0, nullptr, 0.0, -1);
    gemm_big(B, st, B.T1, B.X, B.W1, 1.0, nullptr, 0.0, -1);
    launch_symmetrize(st, B.nblk, B.d_blk, B.d_flags, B.W1, B.W1, nskip);
  }
}

// B^T(y) for every active system; phase-I systems use B'^T (lift + t D).
// With G given (phase-unaware callers excluded), also G = C - B^T(y) + Z.
static void op_BT(Batch& B, hipStream_t st, const double* yv, double* out, bool phase_aware = true,
                  double* G = nullptr) {
  const size_t m0 = B.prof.mark();
  const double* ybase = yv;
  if (phase_aware && B.any_phase1) {
    launch_lift(st, B.S, B.d_sys, B.d_flags, yv, B.ylift);
    ybase = B.ylift;
  }
  // the small-block epilogue's G would miss the phase-I term added below
  double* Gs = (G && !(phase_aware && B.any_phase1)) ? G : nullptr;
  if (B.nmax_small) launch_BT_small(st, B.nblk, B.d_blk, B.d_sys, B.d_flags, ybase, out, B.Cf, B.Z, Gs);
  if (B.maxn > kSmallN) {
    const int nskip = B.nmax_small ? kSmallN : 0;
    launch_form_P(st, B.totL0, B.d_sys, B.d_flags, B.d_ownP, B.S, ybase, B.Pm, nskip);
    launch_BT_pblk(st, B.npblk, B.d_pblk, B.d_sys, B.d_flags, B.Pm, out, nskip);
    launch_BT_dblk(st, B.ndblk, B.d_dblk, B.d_sys, B.d_flags, B.Pm, out, B.nmin_big, gemm_tiles(B.maxn));
  }
  if (phase_aware && B.any_phase1) launch_sub_tD(st, B.nblk, B.d_blk, B.d_sys, B.d_flags, yv, out);
  if (G && !Gs) launch_make_G(st, B.nblk, B.d_blk, B.d_flags, B.Cf, out, B.Z, G, 0);
  else if (G && B.maxn > kSmallN)
    launch_make_G(st, B.nblk, B.d_blk, B.d_flags, B.Cf, out, B.Z, G, B.nmax_small ? kSmallN : 0);
  B.prof.add(PSDP_PROF_BT, m0, B.prof.mark());
}

// B(W) - asub * a; W must be symmetric (callers symmetrise first; B(W) =
// B(sym W)).  Phase-I systems get B'(W) - asub * a'.
static void op_B(Batch& B, hipStream_t st, const double* W, double* out, double asub,
                 bool phase_aware = true) {
  const size_t m0 = B.prof.mark();
  if (B.nmax_small)
    launch_B_small(st, B.totL0, B.d_sys, B.d_flags, B.d_ownP, B.S, W, out, asub);
  if (B.maxn > kSmallN) {
    launch_B_Y(st, B.npairs, B.d_pairs, B.d_sys, B.d_flags, W, B.arena, B.d_blk, B.nmin_big,
               gemm_tiles(B.maxn));
    launch_B_reduce(st, B.totK, B.d_sys, B.d_flags, B.d_ownK, B.S, B.d_pairs, W, B.arena, B.d_blk,
                    out, asub, B.nmax_small ? kSmallN : 0);
  }
  if (phase_aware && B.any_phase1) launch_B_phase1(st, B.S, B.d_sys, B.d_flags, B.d_blk, W, out, asub);
  B.prof.add(PSDP_PROF_B, m0, B.prof.mark());
}

static void op_schur(Batch& B, hipStream_t st) {
  const size_t m0 = B.prof.mark();
  if (B.nmax_small) {
    launch_pre12_small(st, B.npairs, B.nmax_small, B.d_pairs, B.d_sys, B.d_flags, B.Zi, B.X, B.arena,
                       B.d_blk, B.d_offA1);
    launch_pre34_small(st, B.nq2, B.nmax_small, B.d_q2, B.d_sys, B.d_flags, B.arena);
  }
  if (B.maxn > kSmallN) {
    launch_pre12(st, B.npairs, B.d_pairs, B.d_sys, B.d_flags, B.Zi, B.X, B.arena, B.d_blk, B.d_offA1,
                 B.nmin_big, gemm_tiles(B.maxn));
    launch_pre34(st, B.nq2, B.d_q2, B.d_sys, B.d_flags, B.arena, B.nmin_big, gemm_tiles(B.maxn));
  }
  const size_t m1 = B.prof.mark();
  launch_assemble_pair(st, B.nptiles, B.maxn_pair, B.d_ptiles, B.d_terms, B.d_sys, B.d_flags,
                       B.arena, B.Lam, B.prec, B.rscr);
  launch_assemble_grp(st, B.ntiles, B.d_tiles, B.d_terms, B.d_sys, B.d_flags, B.d_gpinfo, B.arena,
                      B.Lam, B.d_gpoff, B.prec);
  const size_t m2 = B.prof.mark();
  B.prof.add(PSDP_PROF_PRE, m0, m1);
  B.prof.add(PSDP_PROF_ASSEMBLE, m1, m2);
  if (B.any_phase1) {
    // phase-I: v = B(D Z^-1 X) and the rank-2 + border transform
    launch_gemm_scaled(st, B.nblk, B.d_blk, B.d_sys, B.d_flags, B.Zi, B.X, B.W1, gemm_tiles(B.maxn));
    launch_symmetrize(st, B.nblk, B.d_blk, B.d_flags, B.W1, B.W1);
    op_B(B, st, B.W1, B.vtmp, 0.0, false);
    launch_lam_phase1(st, B.S, B.maxK, B.d_sys, B.d_flags, B.d_blk, B.W1, B.vtmp, B.Lam);
    B.prof.add(PSDP_PROF_PHASE1, m2, B.prof.mark());
  }
}

// inverses of the factor's diagonal blocks used by the grouped solves (timed
// with the solves)
static void op_ginv(Batch& B, hipStream_t st) {
  if (B.gin.tot[0] > 0) {
    const size_t m0 = B.prof.mark();
    int l = 0;
    for (int m = 1; m < kSG; m *= 2, ++l) {
      const int f = B.gin.first[l];
      for (int ph = 0; ph < 2; ++ph)
        launch_trsv_ginv(st, B.d_sys, B.d_flags, B.d_gin_sys + f, B.d_gin_pre + f, B.gin.cnt[l], B.gin.tot[l],
                         B.Lam, B.Linv, B.Ginv, m, ph);
    }
    const int f = B.gin.first[l];
    launch_trsv_gfinish(st, B.d_sys, B.d_flags, B.d_gin_sys + f, B.d_gin_pre + f, B.gin.cnt[l], B.gin.tot[l],
                        B.Linv, B.Ginv);
    B.prof.add(PSDP_PROF_TRSV, m0, B.prof.mark());
  }
}

static int op_factor(Batch& B, hipStream_t st) {
  B.side_pending = false;
  for (int p = 0; p < B.maxP; ++p) {
    const int f = B.pan.first[p];
    const size_t m0 = B.prof.mark();
    launch_chol_diag(st, B.d_sys, B.d_flags, B.Lam, B.Ldiag, B.Linv, B.d_pan_sys + f, B.pan.cnt[p], p);
    const int f2 = B.trs.first[p];
    launch_chol_trsm(st, B.d_sys, B.d_flags, B.Lam, B.Linv, B.d_trs_sys + f2, B.d_trs_pre + f2,
                     B.trs.cnt[p], B.trs.tot[p], p);
    const size_t m1 = B.prof.mark();
    B.prof.add(PSDP_PROF_CHOL_PANEL, m0, m1);
    if (B.upd.tot[p] > 0) {
      const int g = B.upd.first[p];
      launch_chol_update(st, B.d_sys, B.d_flags, B.Lam, B.Ldiag, B.Linv, B.d_upd_sys + g, B.d_upd_pre + g,
                         B.upd.cnt[p], B.upd.tot[p], p);
    }
    if (B.mid.tot[p] > 0) {
      const int g = B.mid.first[p];
      launch_chol_update_wide(st, B.d_sys, B.d_flags, B.Lam, B.d_mid_sys + g, B.d_mid_pre + g,
                              B.mid.cnt[p], B.mid.tot[p], p, 1);
    }
    if (B.wide.tot[p] > 0) {
      const int g = B.wide.first[p];
      launch_chol_update_wide(st, B.d_sys, B.d_flags, B.Lam, B.d_wide_sys + g, B.d_wide_pre + g,
                              B.wide.cnt[p], B.wide.tot[p], p, 0);
    }
    if (B.lw1.tot[p] > 0 || B.lw2.tot[p] > 0) {
      // the previous side update covers this one's tiles
      if (B.side_pending) PSDP_HIP(hipStreamWaitEvent(st, B.ev_join, 0));
      B.side_pending = false;
      if (B.lw2.tot[p] > 0) {
        const int g = B.lw2.first[p];
        PSDP_HIP(hipEventRecord(B.ev_fork, st));
        PSDP_HIP(hipStreamWaitEvent(B.side, B.ev_fork, 0));
        launch_chol_update_wide(B.side, B.d_sys, B.d_flags, B.Lam, B.d_lw2_sys + g, B.d_lw2_pre + g,
                                B.lw2.cnt[p], B.lw2.tot[p], p, 3);
        PSDP_HIP(hipEventRecord(B.ev_join, B.side));
        B.side_pending = true;
      }
      if (B.lw1.tot[p] > 0) {
        const int g = B.lw1.first[p];
        launch_chol_update_wide(st, B.d_sys, B.d_flags, B.Lam, B.d_lw1_sys + g, B.d_lw1_pre + g,
                                B.lw1.cnt[p], B.lw1.tot[p], p, 2);
      }
    }
    if (B.upd.tot[p] > 0 || B.mid.tot[p] > 0 || B.wide.tot[p] > 0 || B.lw1.tot[p] > 0 || B.lw2.tot[p] > 0)
      B.prof.add(PSDP_PROF_CHOL_UPDATE, m1, B.prof.mark());
    if (B.fus.tot[p] > 0) {
      const int g = B.fus.first[p];
      const size_t m2 = B.prof.mark();
      launch_chol_fused(st, B.d_sys, B.d_flags, B.Lam, B.Ldiag, B.Linv, B.PB, B.d_fus_sys + g, B.d_fus_pre + g,
                        B.fus.cnt[p], B.fus.tot[p], p);
      B.prof.add(PSDP_PROF_CHOL_UPDATE, m2, B.prof.mark());
    }
    if (B.lah.tot[p] > 0) {
      const int gh = B.lah.first[p], gl = B.lal.first[p];
      const size_t m2 = B.prof.mark();
      launch_chol_look(st, B.d_sys, B.d_flags, B.Lam, B.Ldiag, B.Linv, B.d_lah_sys + gh, B.d_lah_pre + gh,
                       B.lah.cnt[p], B.lah.tot[p], B.d_lal_sys + gl, B.d_lal_pre + gl, B.lal.cnt[p],
                       B.lal.tot[p], p);
      B.prof.add(PSDP_PROF_CHOL_UPDATE, m2, B.prof.mark());
    }
    if (B.lft.tot[p] > 0) {
      const int g = B.lft.first[p];
      const size_t m2 = B.prof.mark();
      launch_chol_left(st, B.d_sys, B.d_flags, B.Lam, B.Ldiag, B.Linv, B.d_lft_sys + g, B.d_lft_pre + g,
                       B.lft.cnt[p], B.lft.tot[p], p);
      B.prof.add(PSDP_PROF_CHOL_UPDATE, m2, B.prof.mark());
    }
  }
  if (B.side_pending) {
    const size_t m0 = B.prof.mark();
    PSDP_HIP(hipStreamWaitEvent(st, B.ev_join, 0));
    B.side_pending = false;
    B.prof.add(PSDP_PROF_CHOL_UPDATE, m0, B.prof.mark());
  }
  op_ginv(B, st);
  return PSDP_OK;
}

static int op_solve(Batch& B, hipStream_t st, const double* rhs, double* x) {
  const size_t m0 = B.prof.mark();
  launch_trsv_small(st, (int)B.small_ids.size(), B.d_sys, B.d_flags, B.d_small, B.Lam, B.Linv, rhs, x);
  if (B.small_ids.size() < (size_t)B.S) {
    // forward: z_q = G_q r_q, then the rows below; backward: x_q = G_q^T z_q,
    // then the columns left (r, z scratch; x written group by group)
    PSDP_HIP(hipMemcpyAsync(B.r, rhs, B.totvec * 8, hipMemcpyDeviceToDevice, st));
    for (int q = 0; q < B.maxNG; ++q) {
      const int a = B.gap.first[q];
      launch_trsv_gapply(st, B.d_sys, B.d_flags, B.d_gap_sys + a, B.d_gap_pre + a, B.gap.cnt[q], B.gap.tot[q],
                         B.Ginv, B.r, B.z, q, 0);
      const int f = B.gfu.first[q];
      launch_trsv_gfwd(st, B.d_sys, B.d_flags, B.d_gfu_sys + f, B.d_gfu_pre + f, B.gfu.cnt[q],
                       B.gfu.tot[q], B.Lam, B.z, B.r, q);
    }
    for (int q = B.maxNG - 1; q >= 0; --q) {
      const int a = B.gap.first[q];
      launch_trsv_gapply(st, B.d_sys, B.d_flags, B.d_gap_sys + a, B.d_gap_pre + a, B.gap.cnt[q], B.gap.tot[q],
                         B.Ginv, B.z, x, q, 1);
      const int f = B.gbu.first[q];
      launch_trsv_gbwd(st, B.d_sys, B.d_flags, B.d_gbu_sys + f, B.d_gbu_pre + f, B.gbu.cnt[q],
                       B.gbu.tot[q], B.Lam, x, B.z, q);
    }
  }
  B.prof.add(PSDP_PROF_TRSV, m0, B.prof.mark());
  return PSDP_OK;
}

// Newton solve with iterative refinement (Section IV-A: Lambda v is
// B(Z^-1 B^T(v) X), the Schur complement applied without forming it):
// x = F^{-1} rhs, then up to ir_max corrections x += F^{-1} r with
// r = rhs - Lambda x in FP64.  Each system leaves the loop (parked) once its
// residual is accepted or stops falling; in the precision form the systems
// assembled in FP64 are parked from the start.  first = the iteration's first
// solve.  Scratch: S1, T1, W1 (block arrays free during the solves), BX, vtmp.
static int op_solve_refined(Batch& B, hipStream_t st, const double* rhs, double* x, bool first) {
  int rc = op_solve(B, st, rhs, x);
  // systems factored with a shift are refined against the unshifted product
  const int irm = B.shift_pass ? std::max(B.ir_max, kIrShift) : B.ir_max;
  if (rc || irm == 0) return rc;
  // refinement of every system only when the caller asked for it in FP64
  if (B.f32 || B.ir_max == 0) launch_park(st, B.S, B.d_flags, 0);
  for (int k = 0; k <= irm; ++k) {
    op_BT(B, st, x, B.S1);
    op_sym_ZAX(B, st, B.S1);
    op_B(B, st, B.W1, B.BX, 0.0);
    launch_vec_axpby(st, B.S, B.d_sys, B.d_flags, -1.0, B.BX, 1.0, rhs);   // r = rhs - Lambda x
    launch_ir_check(st, B.S, B.d_sys, B.d_flags, B.BX, rhs, B.d_sc, k, irm, first ? 1 : 0);
    if (k == irm) break;
    if ((rc = op_solve(B, st, B.BX, B.vtmp))) break;
    launch_vec_axpby(st, B.S, B.d_sys, B.d_flags, 1.0, x, 1.0, B.vtmp);
  }
  launch_park(st, B.S, B.d_flags, 1);
  return rc;
}

// identity blocks, C blocks, zeroed Schur matrices with identity padding
static int init_state(Batch& B, hipStream_t st) {
  launch_init_blocks(st, B.nblk, B.d_blk, B.d_sys, B.X, B.Z, B.Cf);
  PSDP_HIP(hipMemsetAsync(B.y, 0, B.totvec * 8 * 10, st));   // all ten vectors
  PSDP_HIP(hipMemsetAsync(B.Lam, 0, B.totlam * 8, st));
  launch_pad_identity(st, B.S, B.d_sys, B.Lam);
  PSDP_HIP(hipGetLastError());
  PSDP_HIP(hipStreamSynchronize(st));
  return PSDP_OK;
}

struct RunState {
  int max_iter = 0;             // iteration cap of this system's run
  int retries = 0;              // passes that repeated a failed Newton step (not iterations)
  int shifts = 0;               // Newton steps whose Schur factorisation needed a shift
  double shf = 0.0;             // shift factor of the next factorisation (0: none)
  int label_iter = -1;          // iteration whose iterate was recorded as the label
  std::vector<double> label_y, label_logx;
  int reason = PSDP_R_MAXITER;
  int iterations = 0;
  bool running = true;
  std::vector<double> dinf_hist;
  int it32 = 0;           // iterations assembled in reduced precision
  int ir_steps = 0;       // refinement corrections applied
  double eta_max = 0.0;   // largest first refinement residual ratio among them
  double phi = NAN, psi = NAN, gap_abs = NAN, gap_rel = NAN, pinf = NAN, dinf = NAN;
};

static void set_flags(Batch& B, const std::vector<RunState>& rs, int* hf) {
  B.shift_pass = false;
  for (int s = 0; s < B.S; ++s) {
    const bool sh = rs[s].running && rs[s].shf > 0.0;
    hf[s] = rs[s].running ? F_ACTIVE | F_CHOLSEL | (B.f32 && !B.asm64[s] ? F_ASM32 : 0) |
                                (sh ? F_SHIFTED : 0)
                          : 0;
    B.h_shf[s] = sh ? rs[s].shf : 0.0;
    B.shift_pass = B.shift_pass || sh;
  }
}

// Idle solver streams, kept per device (creating and destroying a stream
// costs about a tenth of a millisecond each).

// Private solver stream, started after the caller's stream (default priority).
struct SolveStream {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  int dev = 0;
  int open(hipStream_t caller) {
    PSDP_HIP(hipGetDevice(&dev));
    if (!(st = pool_take(dev))) return fail(PSDP_EDEVICE, "stream creation failed");
    PSDP_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    PSDP_HIP(hipEventRecord(ev, caller));
    PSDP_HIP(hipStreamWaitEvent(st, ev, 0));
    return PSDP_OK;
  }
  ~SolveStream() {
    if (st) pool_give(dev, st);
    if (ev) hipEventDestroy(ev);
  }
};

// A captured sequence of launches (hipGraph) replayed once per iteration.
// Capture happens on first use; if the runtime refuses it the sequence runs
// eagerly from then on.  Event pairs recorded by the profiler inside the
// sequence are replayed with it.
struct GraphRun {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  bool failed = false;
  std::vector<std::array<size_t, 3>> pairs;
  ~GraphRun() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
  }
};

template <class F>
static int replay(Batch& B, hipStream_t st, GraphRun& g, F&& fn) {
  // HIP events recorded by graph nodes carry no timestamps, so the
  // per-class profiler runs the launches eagerly
  if (!B.use_graph || g.failed || B.prof.on) return fn();
  if (!g.exec) {
    static const bool dbg = std::getenv("PSDP_GRAPH_DEBUG") != nullptr;
    const size_t p0 = B.prof.pend.size();
    B.prof.fresh(1024 + 8 * (size_t)B.maxP);
    hipError_t eb = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
    if (eb != hipSuccess) {
      if (dbg) std::fprintf(stderr, "graph: begin capture: %s\n", hipGetErrorString(eb));
      (void)hipGetLastError();
      g.failed = true;
      return fn();
    }
    const int rc = fn();
    hipGraph_t gr = nullptr;
    const hipError_t ec = hipStreamEndCapture(st, &gr);
    hipError_t ei = hipSuccess;
    if (rc == PSDP_OK && ec == hipSuccess && gr) ei = hipGraphInstantiate(&g.exec, gr, nullptr, nullptr, 0);
    if (rc != PSDP_OK || ec != hipSuccess || !gr || ei != hipSuccess) {
      if (dbg)
        std::fprintf(stderr, "graph: capture failed (body %d: %s; end %s; instantiate %s)\n", rc,
                     rc ? psdp_last_error() : "", hipGetErrorString(ec), hipGetErrorString(ei));
      (void)hipGetLastError();
      if (gr) hipGraphDestroy(gr);
      g.exec = nullptr;
      g.failed = true;
      B.prof.pend.resize(p0);
      B.prof.fresh(1024 + 8 * (size_t)B.maxP);
      return fn();
    }
    g.graph = gr;
    g.pairs.assign(B.prof.pend.begin() + p0, B.prof.pend.end());
    B.prof.pend.resize(p0);
    B.prof.base = B.prof.next;   // the graph's events stay reserved
  }
  PSDP_HIP(hipGraphLaunch(g.exec, st));
  ++B.graph_launches;
  B.prof.pend.insert(B.prof.pend.end(), g.pairs.begin(), g.pairs.end());
  return PSDP_OK;
}

// One interior-point run of every system marked running.
static int run_ipm(Batch& B, const psdp_opts& o, hipStream_t st, std::vector<RunState>& rs,
                   std::vector<std::vector<psdp_iter_rec>>* hist) {
  const int S = B.S;
  // pinned buffers: the uploads of hf need no wait (hf is rewritten only
  // after the next synchronisation), the read-backs are plain DMA
  int* hf = B.h_hf;
  int* prev = B.h_prev;
  double* hsc = B.h_sc;
  const size_t nsc = (size_t)S * kNSC;
  const int stall_w = 10;
  std::vector<char> was32(S, 0);   // the previous iteration assembled in FP32
  std::vector<char> prev_fail(S, 0);
  std::vector<char> retry(S, 0);   // this pass repeats the previous (failed) Newton step
  std::vector<char> was_shift(S, 0);   // the previous Newton step was factored with a shift
  for (auto& r : rs) r.shf = r.running ? o.chol_shift_force : 0.0;
  // One synchronisation per iteration: after the residual kernels the host
  // reads the scalars and the flags (which still carry the failure bits of
  // the previous Newton step and of this iteration's Z^-1), decides, and
  // uploads the flags of the Newton step without waiting.
  set_flags(B, rs, hf);
  PSDP_HIP(hipMemcpyAsync(B.d_flags, hf, S * 4, hipMemcpyHostToDevice, st));
  // FP64 runs enqueue the next Schur assembly right behind the read-backs
  // and wait only for those (an event), so the host's decisions overlap the
  // assembly; it uses the flags of the previous step, which only adds the
  // assembly of a system that is about to stop.  (The precision form decides
  // each step's assembly precision on the host, and the class profiler
  // needs every launch of a class in one place, so both keep the plain
  // order.)
  const bool hoist = !B.f32 && !B.prof.on && !B.ext;
  hipEvent_t ev_rb = nullptr;
  if (hoist) PSDP_HIP(hipEventCreateWithFlags(&ev_rb, hipEventDisableTiming));
  struct EvGuard {
    hipEvent_t e;
    ~EvGuard() { if (e) hipEventDestroy(e); }
  } ev_guard{ev_rb};
  // the graphs are destroyed before the event above, and only once nothing
  // launched here is still running (the last hoisted assembly may be)
  GraphRun g1, g2, g2s, g3;
  struct Drain {
    hipStream_t s;
    ~Drain() { hipStreamSynchronize(s); }
  } drain{st};
  for (int it = 0;; ++it) {
    // residuals, objectives and the scalars the host decides on
    auto part1 = [&]() -> int {
    { const size_t pm_ = B.prof.mark();
    launch_cholinv(st, B.nblk, B.maxn, B.nmax_small, B.d_blk, B.d_flags, B.Z, B.Zi);
      B.prof.add(PSDP_PROF_CHOLINV, pm_, B.prof.mark()); }
    op_BT(B, st, B.y, B.S1, true, B.G);
    op_B(B, st, B.X, B.BX, 0.0);
    { const size_t pm_ = B.prof.mark();
    launch_block_red(st, B.nblk, B.d_blk, B.d_flags, B.Cf, B.X, B.Z, B.G, B.d_red);
      B.prof.add(PSDP_PROF_MISC, pm_, B.prof.mark()); }
    { const size_t pm_ = B.prof.mark();
    launch_sys_finalize(st, S, B.d_sys, B.d_flags, B.d_red, B.y, B.BX, o.sigma, B.d_sc);
      B.prof.add(PSDP_PROF_MISC, pm_, B.prof.mark()); }
    PSDP_HIP(hipGetLastError());
    PSDP_HIP(hipMemcpyAsync(hsc, B.d_sc, nsc * 8, hipMemcpyDeviceToHost, st));
    PSDP_HIP(hipMemcpyAsync(prev, B.d_flags, S * 4, hipMemcpyDeviceToHost, st));
      return PSDP_OK;
    };
    int rc = replay(B, st, g1, part1);
    if (rc) return rc;
    if (hoist) {
      PSDP_HIP(hipEventRecord(ev_rb, st));
      if ((rc = replay(B, st, g3, [&]() -> int { op_schur(B, st); return PSDP_OK; }))) return rc;
      PSDP_HIP(hipEventSynchronize(ev_rb));
    } else {
      PSDP_HIP(hipStreamSynchronize(st));
    }
    B.prof.harvest();
    if (it > 0) {
      // failure bits of the previous Newton step (a failed step left the
      // iterate unchanged, so this pass can repeat it)
      for (int s = 0; s < S; ++s) {
        was32[s] = (prev[s] & F_ASM32) != 0;
        prev_fail[s] = (prev[s] & F_LAMFAIL) != 0;
        was_shift[s] = (prev[s] & F_SHIFTED) != 0;
        retry[s] = 0;
        RunState& r = rs[s];
        if (!r.running) continue;
        if ((prev[s] & F_LAMFAIL) && (prev[s] & F_ASM32)) {
          // the reduced-precision Schur matrix lost definiteness: the step is
          // repeated with FP64 assembly (same shift)
          B.asm64[s] = 1;
          retry[s] = 1;
        } else if (prev[s] & F_LAMFAIL) {
          // the FP64 factorisation failed: repeat the step with the next
          // shift (the run ends below if it exceeds chol_shift_max)
          r.shf = r.shf > 0.0 ? r.shf * kShiftGrowth : kShiftFirst;
          retry[s] = 1;
        } else {
          if (was_shift[s]) ++r.shifts;
          r.shf = o.chol_shift_force;   // the next step starts unshifted (or at the forced shift)
          if (prev[s] & F_LADDERFAIL) { r.running = false; r.reason = PSDP_R_LADDER; }
        }
        r.retries += retry[s];
      }
    }
    bool any = false;
    for (int s = 0; s < S; ++s) {
      RunState& r = rs[s];
      if (!r.running) continue;
      const double* v = hsc + (size_t)s * kNSC;
      r.phi = v[S_PHI]; r.psi = v[S_PSI]; r.gap_abs = v[S_GAPABS]; r.gap_rel = v[S_GAPREL];
      r.pinf = v[S_PINF]; r.dinf = v[S_DINF];
      // a repeated step sees the same iterate: same scalars, no new iteration
      const int ite = it - r.retries;
      r.iterations = ite;
      if (!retry[s]) r.dinf_hist.push_back(r.dinf);
      // refinement no longer contracts fast: FP64 assembly from here on
      const bool refined = (B.ir_max > 0 && (was32[s] || !B.f32)) || was_shift[s];
      if (it > 0 && refined && !retry[s]) r.ir_steps += (int)v[S_IRSTEPS];
      if (it > 0 && was32[s] && !retry[s]) {
        ++r.it32;
        const double eta = (prev_fail[s] || !(v[S_IRETA] == v[S_IRETA])) ? INFINITY : v[S_IRETA];
        if (B.ir_max > 0) r.eta_max = std::max(r.eta_max, eta);
        if (B.ir_max > 0 && (!(eta <= kIrSwitch) || v[S_IRFAIL] != 0.0)) B.asm64[s] = 1;
      }
      if (hist && !retry[s])
        (*hist)[s].push_back(psdp_iter_rec{ite, r.phi, r.psi, r.gap_rel, r.pinf, r.dinf, v[S_MU], 0, 0});
      const bool finite = std::isfinite(r.phi) && std::isfinite(r.psi) && std::isfinite(r.pinf) &&
                          std::isfinite(r.dinf) && std::isfinite(v[S_TRZX]);
      if ((prev[s] & F_ZFAIL) || !finite) { r.running = false; r.reason = PSDP_R_NONFINITE; continue; }
      const bool ph1 = B.sys[s].mode == 1;
      if (o.stop_rule == PSDP_STOP_ABSOLUTE && !ph1) {
        // the printed test of Section IV-A: the absolute gap alone
        if (r.gap_abs <= o.gap_tol) { r.running = false; r.reason = PSDP_R_CONVERGED; continue; }
      } else {
        const bool gap_ok = r.gap_rel <= o.gap_tol || (ph1 && r.gap_abs <= 1e-2 * o.gap_tol);
        if (gap_ok && r.pinf <= o.feas_tol && r.dinf <= o.feas_tol) {
          r.running = false; r.reason = PSDP_R_CONVERGED; continue;
        }
      }
      if (!ph1) {
        if (r.phi > 0 && v[S_NORMBX] / r.phi <= 1e-6) { r.running = false; r.reason = PSDP_R_FARKAS; continue; }
        // stall: the dual residual, above tolerance, has not fallen 10x in 10 iterations
        if (ite >= stall_w && r.dinf > o.feas_tol && r.dinf > 0.1 * r.dinf_hist[ite - stall_w]) {
          r.running = false; r.reason = PSDP_R_STALL; continue;
        }
      }
      if (ite >= r.max_iter) { r.running = false; r.reason = PSDP_R_MAXITER; continue; }
      // no factorisation left to try for the next Newton step
      if (r.shf > o.chol_shift_max * (1.0 + 1e-12)) { r.running = false; r.reason = PSDP_R_CHOL; continue; }
      any = true;
    }
    // training labels: the iterate at the first iteration with gap_rel <= label_gap
    if (o.label_gap > 0) {
      std::vector<int> want;
      for (int s = 0; s < S; ++s)
        if (rs[s].label_iter < 0 && B.sys[s].mode == 0 && std::isfinite(rs[s].gap_rel) &&
            rs[s].gap_rel <= o.label_gap && !(prev[s] & F_ZFAIL))
          want.push_back(s);
      if (!want.empty()) {
        std::vector<double> yh(B.totvec), lx(B.nblk);
        launch_block_logtrace(st, B.nblk, B.d_blk, B.d_flags, B.X, B.d_red);
        PSDP_HIP(hipMemcpyAsync(yh.data(), B.y, B.totvec * 8, hipMemcpyDeviceToHost, st));
        PSDP_HIP(hipMemcpyAsync(lx.data(), B.d_red, B.nblk * 8, hipMemcpyDeviceToHost, st));
        PSDP_HIP(hipStreamSynchronize(st));
        for (int s : want) {
          const SysDesc& d = B.sys[s];
          rs[s].label_iter = rs[s].iterations;
          rs[s].label_y.assign(yh.begin() + d.voff, yh.begin() + d.voff + d.K);
          rs[s].label_logx.assign(lx.begin() + d.blk0, lx.begin() + d.blk0 + d.nb);
        }
      }
    }
    if (!any) break;
    set_flags(B, rs, hf);
    // the Newton step: Schur complement, factor, solves, directions, steps
    auto part2 = [&]() -> int {
    PSDP_HIP(hipMemcpyAsync(B.d_flags, hf, S * 4, hipMemcpyHostToDevice, st));
    if (B.shift_pass) PSDP_HIP(hipMemcpyAsync(B.d_shf, B.h_shf, S * 8, hipMemcpyHostToDevice, st));
    // ---- Newton system (Alg. 2 processors/root step 1)
    if (!hoist) op_schur(B, st);
    if (B.shift_pass) {
      const size_t pm_ = B.prof.mark();
      launch_schur_shift(st, S, B.d_sys, B.d_flags, B.d_shf, B.Lam, B.d_sc);
      B.prof.add(PSDP_PROF_MISC, pm_, B.prof.mark());
    }
    if (int rc = op_factor(B, st)) return rc;
    // blocks of order <= kSmallN take the fused chains, larger ones the
    // separate products and elementwise kernels (which skip the former)
    const int nskip = B.nmax_small ? kSmallN : 0;
    // Omega_1 = B(Z^-1 G X) - a
    { const size_t pm_ = B.prof.mark();
    op_sym_ZAX(B, st, B.G);
      B.prof.add(PSDP_PROF_GEMM, pm_, B.prof.mark()); }
    op_B(B, st, B.W1, B.rv1, 1.0);
    op_solve_refined(B, st, B.rv1, B.dyh, true);
    // predictor directions (processors step 2) and the corrector right-hand
    // side W = mu Z^-1 - Z^-1 dZ^ dX^
    op_BT(B, st, B.dyh, B.S1);
    { const size_t pm_ = B.prof.mark();
    if (B.nmax_small)
      launch_pred_dir_small(st, B.nblk, B.nmax_small, B.d_blk, B.d_flags, B.d_sc, B.S1, B.G, B.Zi, B.X,
                            B.dZh, B.dXh, B.Wc, B.W1);
    if (B.maxn > kSmallN) {
      launch_axpby(st, B.nblk, B.d_blk, B.d_flags, -1.0, B.G, 1.0, B.S1, B.dZh, nskip);
      gemm_big(B, st, B.Zi, B.dZh, B.T1, 1.0, nullptr, 0.0, -1);
      gemm_big(B, st, B.T1, B.X, B.dXh, -1.0, B.X, -1.0, -1);
      gemm_big(B, st, B.T1, B.dXh, B.Wc, -1.0, B.Zi, 1.0, S_MU);
      launch_symmetrize(st, B.nblk, B.d_blk, B.d_flags, B.Wc, B.W1, nskip);
    }
      B.prof.add(PSDP_PROF_GEMM, pm_, B.prof.mark()); }
    if (o.sigma_rule == PSDP_SIGMA_MEHROTRA) {
      // Mehrotra's sigma from the predictor's step lengths; T1 = sym dX^
      const size_t pm_ = B.prof.mark();
      launch_symmetrize(st, B.nblk, B.d_blk, B.d_flags, B.dXh, B.T1, 0);
      launch_ladder2(st, B.nblk, B.maxn, B.nmax_small, B.d_blk, B.d_flags, B.X, B.T1, B.Z, B.dZh,
                     o.ladder_rho, o.step_frac, o.ladder_len, B.d_kout, B.d_kout + B.nblk);
      launch_mehrotra(st, S, B.nblk, B.d_sys, B.d_blk, B.d_flags, B.d_kout, B.d_kout + B.nblk,
                      o.ladder_rho, o.sigma, B.X, B.T1, B.Z, B.dZh, B.Zi, B.d_red, B.d_sc, B.Wc, B.W1);
      B.prof.add(PSDP_PROF_LADDER, pm_, B.prof.mark());
    }
    op_B(B, st, B.W1, B.rv2, 0.0);
    op_solve_refined(B, st, B.rv2, B.dyb, false);
    // corrector directions (processors step 3), summed with the predictor's
    op_BT(B, st, B.dyb, B.dZb);
    { const size_t pm_ = B.prof.mark();
    if (B.nmax_small)
      launch_corr_dir_small(st, B.nblk, B.nmax_small, B.d_blk, B.d_flags, B.Zi, B.dZb, B.X, B.Wc, B.dXh,
                            B.dZh, B.dX, B.dZ);
    if (B.maxn > kSmallN) {
      gemm_big(B, st, B.Zi, B.dZb, B.T1, 1.0, nullptr, 0.0, -1);
      gemm_big(B, st, B.T1, B.X, B.dXb, -1.0, B.Wc, 1.0, -1);
      launch_combine(st, B.nblk, B.d_blk, B.d_flags, B.dXh, B.dXb, B.dX, B.dZh, B.dZb, B.dZ, nskip);
    }
      B.prof.add(PSDP_PROF_GEMM, pm_, B.prof.mark()); }
    // step lengths and update
    // both ladders in one launch, then both step lengths with the y update
    { const size_t pm_ = B.prof.mark();
    launch_ladder2(st, B.nblk, B.maxn, B.nmax_small, B.d_blk, B.d_flags, B.X, B.dX, B.Z, B.dZ, o.ladder_rho,
                   o.step_frac, o.ladder_len, B.d_kout, B.d_kout + B.nblk);
    launch_steps_update_y(st, B.d_sys, S, B.maxK, B.d_flags, B.d_kout, B.d_kout + B.nblk, o.ladder_rho, B.d_sc, B.y,
                          B.dyh, B.dyb);
      B.prof.add(PSDP_PROF_LADDER, pm_, B.prof.mark()); }
    { const size_t pm_ = B.prof.mark();
    launch_update_blocks(st, B.nblk, B.d_blk, B.d_flags, B.d_sc, B.X, B.dX, B.Z, B.dZ);
      B.prof.add(PSDP_PROF_MISC, pm_, B.prof.mark()); }
    PSDP_HIP(hipGetLastError());
      return PSDP_OK;
    };
    if ((rc = replay(B, st, B.shift_pass ? g2s : g2, part2))) return rc;
    if (hist) {
      PSDP_HIP(hipMemcpyAsync(hsc, B.d_sc, nsc * 8, hipMemcpyDeviceToHost, st));
      PSDP_HIP(hipStreamSynchronize(st));
    B.prof.harvest();
      for (int s = 0; s < S; ++s)
        if (rs[s].running && !(*hist)[s].empty()) {
          (*hist)[s].back().tp = hsc[(size_t)s * kNSC + S_TP];
          (*hist)[s].back().td = hsc[(size_t)s * kNSC + S_TD];
        }
    }
  }
  return PSDP_OK;
}

static void validate_opts(const psdp_opts* in, psdp_opts& o) {
  psdp_opts_default(&o);
  if (in) o = *in;
}

}  // namespace

// ---------------------------------------------------------------------------

// Warm start: y from warm_y, Z projected into the interior, X from warm_logx
// (systems without warm data keep the cold start).
static int warm_project(Batch& B, hipStream_t st, const psdp_opts& o, const std::vector<char>& warm) {
  const int S = B.S;
  std::vector<int> hf(S, 0);
  std::vector<double> yv(B.totvec, 0.0), lx(B.nblk, 0.0);
  for (int s = 0; s < S; ++s) {
    if (!warm[s]) continue;
    hf[s] = F_ACTIVE;
    const SysDesc& d = B.sys[s];
    if (o.warm_y && o.warm_y[s]) std::memcpy(yv.data() + d.voff, o.warm_y[s], d.K * 8);
    for (int j = 0; j < d.nb; ++j)
      lx[d.blk0 + j] = (o.warm_logx && o.warm_logx[s]) ? o.warm_logx[s][j] : 0.0;
  }
  for (double v : lx)
    if (!std::isfinite(v) || std::fabs(v) > 700.0) return fail(PSDP_EINVAL, "warm_logx out of range");
  for (double v : yv)
    if (!std::isfinite(v)) return fail(PSDP_EINVAL, "warm_y is not finite");
  PSDP_HIP(hipMemcpyAsync(B.d_flags, hf.data(), S * 4, hipMemcpyHostToDevice, st));
  PSDP_HIP(hipMemcpyAsync(B.y, yv.data(), B.totvec * 8, hipMemcpyHostToDevice, st));
  PSDP_HIP(hipMemcpyAsync(B.d_red, lx.data(), B.nblk * 8, hipMemcpyHostToDevice, st));
  op_BT(B, st, B.y, B.S1, false);
  launch_axpby(st, B.nblk, B.d_blk, B.d_flags, 1.0, B.S1, -1.0, B.Cf, B.T1);   // W = B^T(y) - C
  launch_certificate(st, B.nblk, B.maxn, B.d_blk, B.d_sys, B.d_flags, B.T1, 60, B.d_cert);
  launch_warm_init(st, B.nblk, B.d_blk, B.d_sys, B.d_flags, B.T1, B.d_cert, B.d_red, o.warm_margin,
                   B.X, B.Z);
  if (o.warm_center) {
    launch_cholinv(st, B.nblk, B.maxn, B.nmax_small, B.d_blk, B.d_flags, B.Z, B.Zi);
    launch_warm_center(st, B.nblk, B.d_blk, B.d_flags, B.Zi, B.d_red, B.X);
  }
  PSDP_HIP(hipGetLastError());
  PSDP_HIP(hipStreamSynchronize(st));
  return PSDP_OK;
}

// ---------------------------------------------------------------------------
// Autotuner: for each block order n with n^2 <= 128 the assembly path (whole
// pairs or grouped tiles) and for each tile count P <= kSmallP the solve path
// (one workgroup per system or groups of tiles) are timed once per process with
// HIP events on up to 8 systems of the batch, and the faster is kept.  Both
// paths of each choice compute the same quantities (they differ in rounding
// order only).
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::pair<int, int>, char> g_tune;   // (0, n) assembly, (1, P) solve -> 1 = pair / one wg

template <class F>
static float time_ms(hipStream_t st, int reps, F&& fn) {
  hipEvent_t a, b;
  hipEventCreate(&a);
  hipEventCreate(&b);
  fn();   // warm-up
  hipEventRecord(a, st);
  for (int i = 0; i < reps; ++i) fn();
  hipEventRecord(b, st);
  hipEventSynchronize(b);
  float ms = 0.f;
  hipEventElapsedTime(&ms, a, b);
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms / reps;
}

static int trial_batch(Batch& T, psdp_sdp* const* sub, int cnt, const Choice& c, hipStream_t st) {
  int rc = build_batch(T, sub, cnt, &c);
  if (rc) return rc;
  if ((rc = init_state(T, st))) return rc;
  std::vector<int> hf(cnt, F_ACTIVE | F_CHOLSEL);
  PSDP_HIP(hipMemcpy(T.d_flags, hf.data(), cnt * 4, hipMemcpyHostToDevice));
  return PSDP_OK;
}

// bucket of the factorisation choice: Schur tile counts 2..3, 4..7, 8..15,
// ... share one (0: a single tile, nothing to choose)
static int sw_bucket(int P) {
  if (P < 2) return 0;
  int b = 0;
  while ((P >> (b + 1)) > 0) ++b;
  return b;
}

// candidates of a bucket, as sw | ssw << 8: left-looking (0) below kLeftMaxP
// tiles, and the super-panel widths where a super-panel fits (sub-panels are
// an explicit option only: at K = 20200 widths 16 in sub-panels of 4 or 8
// took 2.07 and 2.04 s against 2.02 s per certificate without)
static int fact_code(int sw, int ssw) { return (sw < 0 ? 256 + sw : sw) | (ssw << 8); }
static int code_sw(int code) { return (code & 255) >= 253 ? (code & 255) - 256 : code & 255; }
static std::vector<int> sw_candidates(int bucket) {
  std::vector<int> c;
  if ((1 << bucket) < kLeftMaxP) {
    c.push_back(0);                    // left-looking
    c.push_back(fact_code(-2, 0));     // right-looking with the panel solve folded in
    c.push_back(fact_code(-3, 0));     // look-ahead right-looking
  }
  if ((2 << bucket) > 8) {
    c.push_back(fact_code(4, 4));
    c.push_back(fact_code(8, 8));
    c.push_back(fact_code(16, 16));
  } else {
    c.push_back(fact_code(kSW, kSW));
  }
  return c;
}

// the factorisation an option pair asks for: chol_panels -1 = left-looking,
// w > 0 = width w with sub-panels of chol_subpanels (0: none)
static void forced_fact(const psdp_opts& o, int& sw, int& ssw) {
  sw = o.chol_panels == -1 ? 0 : o.chol_panels;
  ssw = o.chol_subpanels > 0 ? o.chol_subpanels : sw;
}

static int tune_choice(psdp_sdp* const* sdps, int count, const psdp_opts& o, hipStream_t st,
                       Choice& ch) {
  ch = default_choice(sdps, count);
  if (o.chol_panels != 0)
    for (int s = 0; s < count; ++s) forced_fact(o, ch.sw[s], ch.ssw[s]);
  for (int s = 0; s < count; ++s) {
    const bool can_pair = pair_ok(sdps[s]);
    const bool can_small = sdps[s]->Kpad / kNB <= kSmallP;
    if (o.asm_path >= 0) ch.pair[s] = can_pair && o.asm_path == 1;
    if (o.solve_path >= 0) ch.small[s] = can_small && o.solve_path == 1;
  }
  for (int kind = 0; kind < 3; ++kind) {
    if (kind == 2 ? o.chol_panels != 0 : (kind == 0 ? o.asm_path : o.solve_path) >= 0) continue;
    std::map<int, std::vector<int>> want;   // key -> systems
    for (int s = 0; s < count; ++s) {
      const int P = (int)(sdps[s]->Kpad / kNB);
      const int key = kind == 0 ? sdps[s]->n : kind == 1 ? P : sw_bucket(P);
      const bool able = kind == 0 ? pair_ok(sdps[s]) : kind == 1 ? key <= kSmallP : key > 0;
      if (!able) continue;
      {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tune.count({kind, key})) continue;
      }
      // trial batches: 8 systems per key for the assembly and solve paths;
      // the factorisation's launches are shared by the whole batch, so its
      // trials take up to 64 (the forms differ in work per launch, which
      // only a batch of the real size weighs against their launch counts)
      if (want[key].size() < (kind == 2 ? 64u : 8u)) want[key].push_back(s);
    }
    for (auto& kv : want) {
      std::vector<psdp_sdp*> sub;
      for (int s : kv.second) sub.push_back(sdps[s]);
      const int cnt = (int)sub.size();
      // candidates: the two paths (kinds 0, 1) or factorisations (kind 2)
      const std::vector<int> widths = kind == 2 ? sw_candidates(kv.first) : std::vector<int>{};
      const int nv = kind == 2 ? (int)widths.size() : 2;
      float t[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
      for (int v = 0; v < nv; ++v) {
        Choice c = default_choice(sub.data(), cnt);
        for (int i = 0; i < cnt; ++i) {
          if (kind == 0) c.pair[i] = (char)v;
          else if (kind == 1) c.small[i] = (char)v;
          else {
            c.sw[i] = code_sw(widths[v]);
            c.ssw[i] = widths[v] >> 8;
          }
        }
        Batch T;
        if (int rc = trial_batch(T, sub.data(), cnt, c, st)) return rc;
        if (kind == 0) {
          t[v] = time_ms(st, 3, [&]() { op_schur(T, st); });
        } else if (kind == 1) {
          // one iteration's share of the path: the grouped path's block
          // inverses and both Newton solves
          op_schur(T, st);
          if (int rc = op_factor(T, st)) return rc;
          t[v] = time_ms(st, 3, [&]() {
            op_ginv(T, st);
            op_solve(T, st, T.rv1, T.dyh);
            op_solve(T, st, T.rv2, T.dyb);
          });
        } else {
          // the assembly restores the matrix the factorisation overwrites
          int frc = PSDP_OK;
          t[v] = time_ms(st, 2, [&]() { op_schur(T, st); if (int rc = op_factor(T, st)) frc = rc; });
          if (frc) return frc;
        }
        PSDP_HIP(hipGetLastError());
      }
      int best = 0;
      for (int v = 1; v < nv; ++v)
        if (t[v] < t[best]) best = v;
      std::lock_guard<std::mutex> lk(g_tune_mu);
      g_tune[{kind, kv.first}] = kind == 2 ? widths[best] : (t[1] <= t[0] ? 1 : 0);
    }
  }
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (int s = 0; s < count; ++s) {
    if (o.asm_path < 0 && pair_ok(sdps[s])) {
      auto it = g_tune.find({0, sdps[s]->n});
      if (it != g_tune.end()) ch.pair[s] = it->second;
    }
    const int P = (int)(sdps[s]->Kpad / kNB);
    if (o.solve_path < 0 && P <= kSmallP) {
      auto it = g_tune.find({1, P});
      if (it != g_tune.end()) ch.small[s] = it->second;
    }
    if (o.chol_panels == 0 && sw_bucket(P) > 0) {
      auto it = g_tune.find({2, sw_bucket(P)});
      if (it != g_tune.end()) {
        ch.sw[s] = code_sw(it->second);
        ch.ssw[s] = it->second >> 8;
      }
    }
  }
  return PSDP_OK;
}

// Device scratch of the allocation-free solve (psdp_ipm_solve_noalloc):
// every table and array of such a solve is carved from this array.  Each
// device holds its own copy until the process ends; the host reaches it only
// through the address hipGetSymbolAddress returns for the current device
// (the array's name in host code is not a device address).  Calls on one
// device share it, so concurrent ones race.
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

static int scratch_ptr(void** out) {
  int dev = 0;
  PSDP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PSDP_EDEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PSDP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return PSDP_OK;
}

// ext (or NULL): device memory that holds every table and array of the
// solve (the allocation-free entry point); the solve then runs eagerly on the
// caller's stream with the default or requested kernel paths, without the
// autotuner, graphs, the class profiler or pinned buffers.
static int solve_core(psdp_sdp* const* sdps, int count, const psdp_opts& o, psdp_result* res,
                      bool use_warm, char* ext = nullptr, size_t ext_bytes = 0) {
  auto t0 = std::chrono::steady_clock::now();
  if (!(o.gap_tol > 0) || !(o.feas_tol > 0) || o.max_iter < 0 || !(o.sigma > 0 && o.sigma < 1) ||
      !(o.step_frac > 0 && o.step_frac <= 1) || !(o.ladder_rho > 0 && o.ladder_rho < 1) ||
      o.ladder_len < 0)
    return fail(PSDP_EINVAL, "invalid solver options");
  if (o.verdict_mode < 0 || o.verdict_mode > 2) return fail(PSDP_EINVAL, "invalid verdict_mode");
  if (o.precision != PSDP_PREC_FP64 && o.precision != PSDP_PREC_FP32 &&
      o.precision != PSDP_PREC_BF16)
    return fail(PSDP_EINVAL, "invalid precision");
  if (o.ir_max > 50) return fail(PSDP_EINVAL, "ir_max above 50");
  if (!(o.chol_shift_max >= 0.0 && o.chol_shift_max < 1.0) ||
      !(o.chol_shift_force >= 0.0 && o.chol_shift_force < 1.0))
    return fail(PSDP_EINVAL, "chol_shift_max and chol_shift_force must lie in [0, 1)");
  if (o.stop_rule != PSDP_STOP_RELATIVE && o.stop_rule != PSDP_STOP_ABSOLUTE)
    return fail(PSDP_EINVAL, "invalid stop_rule");
  if (o.sigma_rule != PSDP_SIGMA_FIXED && o.sigma_rule != PSDP_SIGMA_MEHROTRA)
    return fail(PSDP_EINVAL, "invalid sigma_rule");
  if (o.chol_panels < -3 || o.chol_panels > 32)
    return fail(PSDP_EINVAL, "chol_panels must lie in [-3, 32]");
  if (o.chol_subpanels < 0 || (o.chol_subpanels > 0 && (o.chol_panels <= 0 || o.chol_panels % o.chol_subpanels)))
    return fail(PSDP_EINVAL, "chol_subpanels must divide a chol_panels width (0: none)");
  // all work runs on a private stream (capturable into graphs) ordered
  // after the caller's stream; the allocation-free solve uses the caller's
  SolveStream ss;
  hipStream_t st = (hipStream_t)o.stream;
  if (!ext) {
    if (int rc0 = ss.open((hipStream_t)o.stream)) return rc0;
    st = ss.st;
  }
  Batch B;
  B.ext = ext;
  B.ext_bytes = ext_bytes;
  B.use_graph = o.use_graph != 0 && !ext;
  B.prec = o.precision;
  B.f32 = o.precision != PSDP_PREC_FP64;
  B.asm64.assign(count, 0);
  B.ir_max = o.ir_max >= 0 ? o.ir_max : (B.f32 ? 6 : 0);
  B.prof.on = o.prof != nullptr && !ext;
  B.prof.st = st;
  B.prof.out = o.prof;
  Choice ch;
  int rc = PSDP_OK;
  if (ext) {
    ch = default_choice(sdps, count);
    for (int s = 0; s < count; ++s) {
      if (o.asm_path >= 0) ch.pair[s] = pair_ok(sdps[s]) && o.asm_path == 1;
      if (o.solve_path >= 0) ch.small[s] = sdps[s]->Kpad / kNB <= kSmallP && o.solve_path == 1;
      if (o.chol_panels != 0) forced_fact(o, ch.sw[s], ch.ssw[s]);
    }
  } else if ((rc = tune_choice(sdps, count, o, st, ch))) {
    return rc;
  }
  if ((rc = build_batch(B, sdps, count, &ch))) return rc;
  if ((rc = init_state(B, st))) return rc;
  std::vector<char> warm(count, 0);
  bool anywarm = false;
  if (use_warm)
    for (int s = 0; s < count; ++s) {
      warm[s] = (o.warm_y && o.warm_y[s]) || (o.warm_logx && o.warm_logx[s]);
      anywarm = anywarm || warm[s];
    }
  auto since = [](std::chrono::steady_clock::time_point a) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - a).count();
  };
  const double t_prep = since(t0);
  auto tw = std::chrono::steady_clock::now();
  if (anywarm && (rc = warm_project(B, st, o, warm))) return rc;
  if (anywarm) PSDP_HIP(hipStreamSynchronize(st));
  const double t_warm = anywarm ? since(tw) : 0.0;
  auto tp = std::chrono::steady_clock::now();
  double t_paper = 0.0, t_ph1 = 0.0;
  std::vector<std::vector<psdp_iter_rec>> hist(count);
  std::vector<double> logx(B.nblk, NAN);
  std::vector<RunState> rs(count);
  for (int s = 0; s < count; ++s)
    rs[s].max_iter = (warm[s] && o.warm_iter_cap > 0) ? std::min(o.max_iter, o.warm_iter_cap) : o.max_iter;
  std::vector<double> y1(B.totvec, 0.0), y2(B.totvec, 0.0);

  // pass 1: the paper's SDP
  if (o.verdict_mode != PSDP_VERDICT_PHASE1_ONLY) {
    if ((rc = run_ipm(B, o, st, rs, o.record_history ? &hist : nullptr))) return rc;
    t_paper = since(tp);
    PSDP_HIP(hipMemcpyAsync(y1.data(), B.y, B.totvec * 8, hipMemcpyDeviceToHost, st));
    {
      std::vector<int> hf(count, F_ACTIVE);
      PSDP_HIP(hipMemcpyAsync(B.d_flags, hf.data(), count * 4, hipMemcpyHostToDevice, st));
      launch_block_logtrace(st, B.nblk, B.d_blk, B.d_flags, B.X, B.d_red);
      PSDP_HIP(hipMemcpyAsync(logx.data(), B.d_red, B.nblk * 8, hipMemcpyDeviceToHost, st));
    }
    PSDP_HIP(hipStreamSynchronize(st));
    B.prof.harvest();
  } else {
    for (auto& r : rs) { r.running = false; r.reason = -1; }
  }

  // pass 2: phase-I margin SDP for the undecided systems
  std::vector<char> need(count, 0);
  bool anyneed = false;
  for (int s = 0; s < count; ++s) {
    if (o.verdict_mode == PSDP_VERDICT_PHASE1_ONLY) need[s] = 1;
    else if (o.verdict_mode == PSDP_VERDICT_PAPER_THEN_PHASE1 && rs[s].reason != PSDP_R_CONVERGED &&
             rs[s].reason != PSDP_R_FARKAS && !warm[s])   // a warm run that fails falls back cold
      need[s] = 1;
    anyneed = anyneed || need[s];
  }
  std::vector<RunState> r1(count);
  for (auto& q : r1) q.max_iter = o.max_iter;
  auto t1p = std::chrono::steady_clock::now();
  if (anyneed) {
    for (int s = 0; s < count; ++s) {
      B.sys[s].mode = need[s] ? 1 : 0;
      r1[s].running = need[s];
    }
    B.any_phase1 = true;
    PSDP_HIP(hipMemcpyAsync(B.d_sys, B.sys.data(), B.sys.size() * sizeof(SysDesc), hipMemcpyHostToDevice, st));
    PSDP_HIP(hipStreamSynchronize(st));
    if ((rc = init_state(B, st))) return rc;
    std::vector<int> hf(count, 0);
    for (int s = 0; s < count; ++s) hf[s] = need[s] ? F_ACTIVE : 0;
    PSDP_HIP(hipMemcpyAsync(B.d_flags, hf.data(), count * 4, hipMemcpyHostToDevice, st));
    launch_phase1_vectors(st, count, B.d_sys, B.d_flags, B.y, B.rv1);
    op_BT(B, st, B.rv1, B.S1, false);                                  // B_K
    launch_axpby(st, B.nblk, B.d_blk, B.d_flags, -1.0, B.S1, 0.0, B.S1, B.Cf);   // C' = -B_K
    PSDP_HIP(hipGetLastError());
    PSDP_HIP(hipStreamSynchronize(st));
    std::vector<std::vector<psdp_iter_rec>> h2(count);
    if ((rc = run_ipm(B, o, st, r1, nullptr))) return rc;
    PSDP_HIP(hipMemcpyAsync(y2.data(), B.y, B.totvec * 8, hipMemcpyDeviceToHost, st));
    PSDP_HIP(hipStreamSynchronize(st));
    B.prof.harvest();
    t_ph1 = since(t1p);
  }
  auto tc = std::chrono::steady_clock::now();

  // verdicts; certificate vectors
  std::vector<double> ycert(B.totvec, 0.0);
  std::vector<int> verdict(count, PSDP_UNKNOWN), wantcert(count, 0);
  std::vector<double> tstar(count, NAN);
  for (int s = 0; s < count; ++s) {
    const SysDesc& d = B.sys[s];
    psdp_sdp* p = sdps[s];
    if (!need[s]) {
      if (rs[s].reason == PSDP_R_CONVERGED) {
        wantcert[s] = 1;
        std::memcpy(ycert.data() + d.voff, y1.data() + d.voff, d.K * 8);
      } else if (rs[s].reason == PSDP_R_FARKAS) {
        verdict[s] = PSDP_INFEASIBLE;
      }
      continue;
    }
    const double* yp = y2.data() + d.voff;
    const double t = yp[d.K - 1];
    tstar[s] = t;
    const RunState& q = r1[s];
    const bool decided = q.reason == PSDP_R_CONVERGED ||
                         (q.reason == PSDP_R_CHOL && std::fabs(t) > q.gap_abs && q.pinf <= 1e-6 &&
                          q.dinf <= 1e-6);
    if (decided && t > 1e-6) {
      // y = (u, 1 - sum u), rescaled so that B^T(y) >= C
      double su = 0.0;
      for (int k = 0; k < d.K - 1; ++k) su += yp[k];
      double cmax = 0.0;
      for (int j = 0; j < d.nb; ++j) cmax = std::max(cmax, p->cdiag_h[j] / p->scale_h[j]);
      const double ratio = cmax / t;
      double* yc = ycert.data() + d.voff;
      for (int k = 0; k < d.K - 1; ++k) yc[k] = yp[k] * ratio;
      yc[d.K - 1] = (-su + 1.0) * ratio;
      wantcert[s] = 1;
    } else if (decided && t < -1e-6) {
      verdict[s] = PSDP_INFEASIBLE;
    }
  }
  std::vector<double> cert((size_t)B.nblk * 2, 0.0);
  bool anycert = false;
  std::vector<int> hf(count, 0);
  for (int s = 0; s < count; ++s) {
    hf[s] = wantcert[s] ? F_ACTIVE : 0;
    anycert = anycert || wantcert[s];
  }
  if (anycert) {
    PSDP_HIP(hipMemcpyAsync(B.d_flags, hf.data(), count * 4, hipMemcpyHostToDevice, st));
    PSDP_HIP(hipMemcpyAsync(B.y, ycert.data(), B.totvec * 8, hipMemcpyHostToDevice, st));
    op_BT(B, st, B.y, B.S1, false);
    const size_t pm0 = B.prof.mark();
    launch_certificate(st, B.nblk, B.maxn, B.d_blk, B.d_sys, B.d_flags, B.S1, 60, B.d_cert);
    B.prof.add(PSDP_PROF_CERT, pm0, B.prof.mark());
    PSDP_HIP(hipGetLastError());
    PSDP_HIP(hipMemcpyAsync(cert.data(), B.d_cert, cert.size() * 8, hipMemcpyDeviceToHost, st));
    PSDP_HIP(hipStreamSynchronize(st));
    B.prof.harvest();
  }
  const double elapsed = since(t0), t_cert = since(tc);
  for (int s = 0; s < count; ++s) {
    psdp_sdp* p = sdps[s];
    const SysDesc& d = B.sys[s];
    psdp_result& R = res[s];
    const RunState& r = rs[s];
    R.reason = r.reason;
    R.iterations = r.iterations;
    R.phi = r.phi; R.psi = r.psi; R.gap_abs = r.gap_abs; R.gap_rel = r.gap_rel;
    R.pinf = r.pinf; R.dinf = r.dinf;
    R.margin = R.margin_P = R.margin_D = NAN;
    R.phase1_used = need[s];
    R.phase1_iterations = need[s] ? r1[s].iterations : 0;
    R.t_star = tstar[s];
    R.time_solve_s = elapsed;
    R.iters_lowprec = r.it32 + (need[s] ? r1[s].it32 : 0);
    R.ir_steps = r.ir_steps + (need[s] ? r1[s].ir_steps : 0);
    R.ir_eta_max = R.iters_lowprec ? std::max(r.eta_max, need[s] ? r1[s].eta_max : 0.0) : NAN;
    R.chol_shifts = r.shifts + (need[s] ? r1[s].shifts : 0);
    R.graph_replays = B.graph_launches;
    R.phase1_reason = need[s] ? r1[s].reason : -1;
    R.chol_panels = B.use_sw[s];
    R.chol_subpanels = B.sys[s].ssw;
    R.time_prepare_s = t_prep;
    R.time_warm_s = t_warm;
    R.time_paper_s = t_paper;
    R.time_phase1_s = t_ph1;
    R.time_cert_s = t_cert;
    R.asm_path = B.use_pair[s] && pair_ok(p);
    R.solve_path = B.use_small[s] && d.P <= kSmallP;
    R.label_iter = r.label_iter;
    if (r.label_iter >= 0) {
      if (R.label_y) std::memcpy(R.label_y, r.label_y.data(), d.K * 8);
      if (R.label_logx) std::memcpy(R.label_logx, r.label_logx.data(), d.nb * 8);
    }
    R.warm_used = warm[s];
    R.warm_fallback = 0;
    R.warm_iterations = warm[s] ? r.iterations : 0;
    if (R.logx)
      for (int j = 0; j < d.nb; ++j) R.logx[j] = logx[d.blk0 + j];
    R.history_len = 0;
    if (R.history && R.history_cap > 0) {
      const int nrec = std::min<int>(R.history_cap, (int)hist[s].size());
      std::memcpy(R.history, hist[s].data(), nrec * sizeof(psdp_iter_rec));
      R.history_len = nrec;
    }
    int v = verdict[s];
    const double* yc = ycert.data() + d.voff;
    if (wantcert[s]) {
      bool pass = true;
      double mg = INFINITY, mP = INFINITY, mD = INFINITY;
      for (int j = 0; j < d.nb; ++j) {
        const double* c = cert.data() + (size_t)(d.blk0 + j) * 2;
        pass = pass && c[0] != 0.0;
        mg = std::min(mg, c[1]);
        if (j < d.L) mP = std::min(mP, c[1]); else mD = std::min(mD, c[1]);
      }
      R.margin = mg; R.margin_P = mP; R.margin_D = mD;
      v = pass ? PSDP_FEASIBLE : PSDP_UNKNOWN;
      if (need[s]) {
        double sum = 0.0;
        for (int k = 0; k < d.K; ++k) sum += yc[k];
        R.phi = NAN; R.psi = sum; R.gap_abs = NAN; R.gap_rel = NAN;
        R.pinf = r1[s].pinf; R.dinf = r1[s].dinf;
      }
    } else if (need[s]) {
      R.phi = R.psi = R.gap_abs = R.gap_rel = NAN;
      R.pinf = r1[s].pinf; R.dinf = r1[s].dinf;
    }
    R.verdict = v;
    const double* yout = need[s] ? yc : y1.data() + d.voff;
    if (R.y) std::memcpy(R.y, yout, d.K * sizeof(double));
    if (R.P) {
      const int n = p->n;
      const bool keep = v == PSDP_FEASIBLE;
      for (int h = 0; h < p->L0; ++h)
        for (int b = 0; b < p->Nt; ++b) {
          const int pp = p->basis.pairs[2 * b], qq = p->basis.pairs[2 * b + 1];
          const double val = keep ? yc[(int64_t)h * p->Nt + b] : 0.0;
          R.P[((int64_t)h * n + pp) * n + qq] = val;
          R.P[((int64_t)h * n + qq) * n + pp] = val;
        }
    }
  }
  return PSDP_OK;
}

int solve_batch(psdp_sdp* const* sdps, int count, const psdp_opts* opts, psdp_result* res, bool noalloc) {
  auto t0 = std::chrono::steady_clock::now();
  psdp_opts o;
  validate_opts(opts, o);
  if (o.warm_iter_cap < 0) return fail(PSDP_EINVAL, "warm_iter_cap < 0");
  if (!(o.warm_margin >= 0.0) || !(o.warm_margin < 1.0)) return fail(PSDP_EINVAL, "warm_margin not in [0, 1)");
  char* ext = nullptr;
  if (noalloc) {
    void* p = nullptr;
    if (int rc0 = scratch_ptr(&p)) return rc0;
    ext = (char*)p;
  }
  int rc = solve_core(sdps, count, o, res, true, ext, kScratchBytes);
  if (rc) return rc;
  // rejected warm starts: solve again from the cold start
  std::vector<int> redo;
  for (int s = 0; s < count; ++s)
    if (res[s].warm_used &&
        (res[s].verdict == PSDP_UNKNOWN || (o.warm_iter_cap > 0 && res[s].iterations > o.warm_iter_cap)))
      redo.push_back(s);
  if (!redo.empty()) {
    std::vector<psdp_sdp*> sub;
    std::vector<psdp_result> rr;
    for (int s : redo) {
      sub.push_back(sdps[s]);
      rr.push_back(res[s]);   // same caller buffers
    }
    if ((rc = solve_core(sub.data(), (int)sub.size(), o, rr.data(), false, ext, kScratchBytes))) return rc;
    for (size_t i = 0; i < redo.size(); ++i) {
      const int wit = res[redo[i]].warm_iterations;
      res[redo[i]] = rr[i];
      res[redo[i]].warm_used = 0;
      res[redo[i]].warm_fallback = 1;
      res[redo[i]].warm_iterations = wit;
    }
  }
  const double el = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  for (int s = 0; s < count; ++s) res[s].time_solve_s = el;
  return PSDP_OK;
}

int eval_newton(psdp_sdp* sdp, const double* X, const double* Z, const double* y, double* Zi,
                double* BTy, double* BX, double* Lam, double* LamL, double* sol, int chol_panels,
                int chol_subpanels, hipStream_t st) {
  Batch B;
  Choice ch = default_choice(&sdp, 1);
  if (chol_panels != 0) {
    ch.sw[0] = chol_panels == -1 ? 0 : chol_panels;
    ch.ssw[0] = chol_subpanels > 0 ? chol_subpanels : ch.sw[0];
  }
  int rc = build_batch(B, &sdp, 1, &ch);
  if (rc) return rc;
  if ((rc = init_state(B, st))) return rc;
  const SysDesc& d = B.sys[0];
  const int64_t nb = sdp->nb, nn = (int64_t)sdp->bo * sdp->bo;
  PSDP_HIP(hipMemcpyAsync(B.X, X, nb * nn * 8, hipMemcpyHostToDevice, st));
  PSDP_HIP(hipMemcpyAsync(B.Z, Z, nb * nn * 8, hipMemcpyHostToDevice, st));
  PSDP_HIP(hipMemcpyAsync(B.y, y, d.K * 8, hipMemcpyHostToDevice, st));
  const int one = F_ACTIVE | F_CHOLSEL;
  PSDP_HIP(hipMemcpyAsync(B.d_flags, &one, 4, hipMemcpyHostToDevice, st));
  launch_cholinv(st, B.nblk, B.maxn, B.nmax_small, B.d_blk, B.d_flags, B.Z, B.Zi);
  op_BT(B, st, B.y, B.S1);
  op_B(B, st, B.X, B.BX, 0.0);
  op_schur(B, st);
  PSDP_HIP(hipGetLastError());
  if (Zi) PSDP_HIP(hipMemcpyAsync(Zi, B.Zi, nb * nn * 8, hipMemcpyDeviceToHost, st));
  if (BTy) PSDP_HIP(hipMemcpyAsync(BTy, B.S1, nb * nn * 8, hipMemcpyDeviceToHost, st));
  if (BX) PSDP_HIP(hipMemcpyAsync(BX, B.BX, d.K * 8, hipMemcpyDeviceToHost, st));
  std::vector<double> full((size_t)d.Kpad * d.Kpad);
  if (Lam) {
    // the assembly builds the lower triangle (all the factorisation reads);
    // the caller gets it mirrored
    PSDP_HIP(hipMemcpyAsync(full.data(), B.Lam, full.size() * 8, hipMemcpyDeviceToHost, st));
    PSDP_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < d.K; ++i)
      for (int j = 0; j < d.K; ++j)
        Lam[(int64_t)i * d.K + j] = j <= i ? full[(size_t)i * d.Kpad + j] : full[(size_t)j * d.Kpad + i];
  }
  if (int rc = op_factor(B, st)) return rc;
  op_solve(B, st, B.y, B.dyh);
  PSDP_HIP(hipGetLastError());
  if (LamL) {
    std::vector<double> dg((size_t)d.P * kNB * kNB);
    PSDP_HIP(hipMemcpyAsync(full.data(), B.Lam, full.size() * 8, hipMemcpyDeviceToHost, st));
    PSDP_HIP(hipMemcpyAsync(dg.data(), B.Ldiag, dg.size() * 8, hipMemcpyDeviceToHost, st));
    PSDP_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < d.K; ++i)
      for (int j = 0; j < d.K; ++j) {
        double v = 0.0;
        if (j <= i) {
          const int ti = i / kNB, tj = j / kNB;
          v = (ti == tj) ? dg[(size_t)ti * kNB * kNB + (i % kNB) * kNB + (j % kNB)]
                         : full[(size_t)i * d.Kpad + j];
        }
        LamL[(int64_t)i * d.K + j] = v;
      }
  }
  if (sol) PSDP_HIP(hipMemcpyAsync(sol, B.dyh, d.K * 8, hipMemcpyDeviceToHost, st));
  int fl = 0;
  PSDP_HIP(hipMemcpyAsync(&fl, B.d_flags, 4, hipMemcpyDeviceToHost, st));
  PSDP_HIP(hipStreamSynchronize(st));
  if (fl & F_ZFAIL) return fail(PSDP_ENUMERIC, "Z is not positive definite");
  if (fl & F_LAMFAIL) return fail(PSDP_ENUMERIC, "the Schur complement is not positive definite");
  return PSDP_OK;
}

int eval_schur(psdp_sdp* sdp, const double* X, const double* Z, int precision, double* Lam,
               hipStream_t st) {
  if (precision != PSDP_PREC_FP64 && precision != PSDP_PREC_FP32 && precision != PSDP_PREC_BF16)
    return fail(PSDP_EINVAL, "invalid precision");
  Batch B;
  B.prec = precision;
  B.f32 = precision != PSDP_PREC_FP64;
  int rc = build_batch(B, &sdp, 1);
  if (rc) return rc;
  if ((rc = init_state(B, st))) return rc;
  const SysDesc& d = B.sys[0];
  const int64_t nb = sdp->nb, nn = (int64_t)sdp->bo * sdp->bo;
  PSDP_HIP(hipMemcpyAsync(B.X, X, nb * nn * 8, hipMemcpyHostToDevice, st));
  PSDP_HIP(hipMemcpyAsync(B.Z, Z, nb * nn * 8, hipMemcpyHostToDevice, st));
  const int one = F_ACTIVE | F_CHOLSEL | (B.f32 ? F_ASM32 : 0);
  PSDP_HIP(hipMemcpyAsync(B.d_flags, &one, 4, hipMemcpyHostToDevice, st));
  launch_cholinv(st, B.nblk, B.maxn, B.nmax_small, B.d_blk, B.d_flags, B.Z, B.Zi);
  op_schur(B, st);
  PSDP_HIP(hipGetLastError());
  std::vector<double> full((size_t)d.Kpad * d.Kpad);
  PSDP_HIP(hipMemcpyAsync(full.data(), B.Lam, full.size() * 8, hipMemcpyDeviceToHost, st));
  int fl = 0;
  PSDP_HIP(hipMemcpyAsync(&fl, B.d_flags, 4, hipMemcpyDeviceToHost, st));
  PSDP_HIP(hipStreamSynchronize(st));
  if (fl & F_ZFAIL) return fail(PSDP_ENUMERIC, "Z is not positive definite");
  for (int i = 0; i < d.K; ++i)
    for (int j = 0; j < d.K; ++j)
      Lam[(int64_t)i * d.K + j] = j <= i ? full[(size_t)i * d.Kpad + j] : full[(size_t)j * d.Kpad + i];
  return PSDP_OK;
}

int eval_ladder(psdp_sdp* sdp, const double* V, const double* dV, const psdp_opts* opts,
                double* step, int* kstar) {
  psdp_opts o;
  validate_opts(opts, o);
  hipStream_t st = (hipStream_t)o.stream;
  Batch B;
  int rc = build_batch(B, &sdp, 1);
  if (rc) return rc;
  const int64_t nb = sdp->nb, nn = (int64_t)sdp->bo * sdp->bo;
  PSDP_HIP(hipMemcpyAsync(B.X, V, nb * nn * 8, hipMemcpyHostToDevice, st));
  PSDP_HIP(hipMemcpyAsync(B.dX, dV, nb * nn * 8, hipMemcpyHostToDevice, st));
  const int one = F_ACTIVE;
  PSDP_HIP(hipMemcpyAsync(B.d_flags, &one, 4, hipMemcpyHostToDevice, st));
  launch_ladder(st, B.nblk, B.maxn, B.nmax_small, B.d_blk, B.d_flags, B.X, B.dX, o.ladder_rho, o.step_frac,
                o.ladder_len, B.d_kout);
  launch_ladder_step(st, B.d_sys, 1, B.d_flags, B.d_kout, o.ladder_rho, S_TP, B.d_sc);
  PSDP_HIP(hipGetLastError());
  std::vector<int> k(B.nblk);
  double t = 0;
  PSDP_HIP(hipMemcpyAsync(k.data(), B.d_kout, B.nblk * 4, hipMemcpyDeviceToHost, st));
  PSDP_HIP(hipMemcpyAsync(&t, B.d_sc + S_TP, 8, hipMemcpyDeviceToHost, st));
  PSDP_HIP(hipStreamSynchronize(st));
  int km = 0;
  for (int v : k) {
    if (v < 0) { km = -1; break; }
    km = std::max(km, v);
  }
  *kstar = km;
  *step = km < 0 ? 0.0 : t;
  return PSDP_OK;
}

}  // namespace psdp
