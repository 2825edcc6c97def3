// Batches of independent SPOD problems: grouped launches (one workgroup per
// work unit, or persistent workgroups that take units from a device queue),
// hipGraph replay and an autotuner over the launch shapes.  The per-problem
// arithmetic is the single-problem path's; only the mapping of workgroups to
// problems differs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "internal.h"

namespace spod {
namespace {

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

struct ProblemSlots {
  Plan* plan = nullptr;
  int n_modes = 0;
  int64_t ldq = 0;   // row stride of the problem's blocks in the workspace (grouped launches)
  size_t ws_qhat = 0, ws_gram = 0, ws_part = 0;                        // workspace offsets
  size_t o_mean = 0, o_lam = 0, o_psi = 0, o_info = 0, o_phi = 0, o_nvalid = 0;  // output offsets
};

struct Group {
  int key = 0;               // nfft (transform) or ceil(L/16) (Gram)
  int chain = 0;             // 0: problems with L <= 32, 1: L > 32
  size_t off = 0;            // byte offset of the item array in the table
  int n = 0, wgs = 0;
  int queue = 0;             // its counter in the batch's queue array (persistent launches)
};

constexpr int NQUEUE = 256;   // work-queue counters (one per grouped launch)

// Problems with more than 32 blocks form a second chain of launches: their
// Gram (64 x 64 tiles) is bound by MFMA issue and their eigensolves by LDS
// latency, while the other chain's transforms and modes are bound by HBM, so
// the two run side by side (a fork onto a second stream, parallel branches of
// the graph).
constexpr int NCHAIN = 2;
int chain_of(const Plan& p) { return p.nblocks > 32 ? 1 : 0; }

}  // namespace

struct Batch {
  std::vector<ProblemSlots> pb;
  spod_precision prec = SPOD_PREC_FP64;
  int device = 0;
  bool grouped = true, use_graph = true, started = false;
  int64_t gram_target = 8192;
  // launch shapes (options, or the autotuner's choice): transform tile (0 =
  // the single-problem default, 16, 32), eigensolver threads (0 = the
  // single-problem rule, 256, 1024), persistent workgroups (0 or 1)
  int fft_tile = 0, eig_threads = 0, persistent = 0;
  int* d_queue = nullptr;    // [NQUEUE] work-queue counters
  int n_queue = 0;           // counters in use
  size_t ws_bytes = 0, out_bytes = 0;

  // work tables (device) and the pointers they were built for
  void* d_table = nullptr;
  size_t table_cap = 0;
  std::vector<const void*> q_built;
  void* out_built = nullptr;
  void* ws_built = nullptr;
  spod_dtype dtype_built = SPOD_F32;
  int64_t target_built = -1;
  int tile_built = -1;
  bool tables_ok = false;
  std::vector<Group> fft_groups, gram_groups, eig_groups;   // eig: by L bucket (16, 32, 64)
  std::vector<int> fft_fallback;                 // problems launched on their own
  Group comb_g[NCHAIN], modes_g[NCHAIN];
  size_t modes_lds = 0;

  hipStream_t cap_stream = nullptr;
  hipStream_t side = nullptr;                    // the second chain
  hipEvent_t fork = nullptr, join = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

bool c128(const Batch& b) { return b.prec == SPOD_PREC_FP64; }
size_t csize(const Batch& b) { return c128(b) ? 16 : 8; }

// The workspace is laid out for the largest Gram split any target may choose.
void layout(Batch& b) {
  const int64_t tmax = std::max<int64_t>(b.gram_target, 16384);
  size_t ws = 0, out = 0;
  for (auto& s : b.pb) {
    const Plan& p = *s.plan;
    const size_t K = p.nfreq, L = p.nblocks, M = p.M;
    // complex64 rows get an even stride, so they are 16-byte aligned for the
    // grouped kernels' vector loads and stores (the pad column is never read)
    s.ldq = c128(b) ? p.M : (p.M + 1) / 2 * 2;
    s.ws_qhat = ws;
    ws += up256(csize(b) * K * L * (size_t)s.ldq);
    s.ws_gram = ws;
    ws += up256(16 * K * L * L);
    s.ws_part = ws;
    const size_t D = (size_t)p.gram_dim;
    const size_t smax = (size_t)gram_split_for(p, tmax);
    ws += up256(16 * K * smax * D * D);
    s.o_mean = out;
    out += up256(8 * M);
    s.o_lam = out;
    out += up256(8 * K * L);
    s.o_psi = out;
    out += up256(16 * K * L * L);
    s.o_info = out;
    out += up256(4 * K);
    s.o_phi = out;
    out += up256(csize(b) * K * (size_t)s.n_modes * M);
    s.o_nvalid = out;
    out += up256(4 * K);
  }
  b.ws_bytes = std::max<size_t>(ws, 256);
  b.out_bytes = std::max<size_t>(out, 256);
}

void drop_graph(Batch& b) {
  if (b.exec) (void)hipGraphExecDestroy(b.exec);
  b.exec = nullptr;
}

void apply_target(Batch& b) {
  for (auto& s : b.pb) plan_set_gram_split(*s.plan, gram_split_for(*s.plan, b.gram_target));
}

bool fused_ok(const Plan& p) {
  return !p.general && p.n_mean_bins >= 0 && p.nfft >= 16 && p.nfft <= 512 &&
         p.step * 2 == p.nfft;
}

template <typename It>
void put(std::vector<char>& host, Group& g, const std::vector<It>& items) {
  while (host.size() % 64) host.push_back(0);
  g.off = host.size();
  g.n = (int)items.size();
  const char* src = reinterpret_cast<const char*>(items.data());
  host.insert(host.end(), src, src + sizeof(It) * items.size());
}

spod_status build_tables(Batch& b, const void* const* q, spod_dtype dtype, char* out, char* ws) {
  std::vector<char> host;
  // transform: grouped by chain and nfft
  std::map<std::pair<int, int>, std::vector<FftItem>> fft;
  b.fft_fallback.clear();
  for (size_t i = 0; i < b.pb.size(); ++i) {
    const ProblemSlots& s = b.pb[i];
    const Plan& p = *s.plan;
    if (!fused_ok(p)) {
      b.fft_fallback.push_back((int)i);
      continue;
    }
    FftItem it{};
    it.q = q[i];
    it.mean = reinterpret_cast<double*>(out + s.o_mean);
    it.window = p.d_window;
    it.tw = c128(b) ? (const void*)p.d_tw64 : (const void*)p.d_tw32;
    it.qhat = ws + s.ws_qhat;
    it.M = p.M;
    it.ldq = s.ldq;
    it.nt = p.nt;
    it.step = (int)p.step;
    it.L = (int)p.nblocks;
    it.kappa = p.kappa;
    it.mb.n = p.n_mean_bins;
    for (int j = 0; j < p.n_mean_bins; ++j) {
      it.mb.k[j] = p.mean_bin[j];
      it.mb.wr[j] = p.what_re[j];
      it.mb.wi[j] = p.what_im[j];
    }
    fft[{chain_of(p), (int)p.nfft}].push_back(it);
  }
  b.fft_groups.clear();
  for (auto& kv : fft) {
    Group g;
    g.chain = kv.first.first;
    g.key = kv.first.second;
    const int T = fft_group_tile(g.key, b.prec, b.fft_tile);
    // the longest workgroups (most blocks) first, so the short ones fill the
    // end of the launch; a workgroup's result does not depend on its place
    std::stable_sort(kv.second.begin(), kv.second.end(),
                     [](const FftItem& x, const FftItem& y) { return x.L > y.L; });
    int64_t start = 0;
    for (auto& it : kv.second) {
      it.start = (int)start;
      start += (it.M + T - 1) / T;
    }
    if (start > 0x7fffffff) return fail(SPOD_ERR_UNSUPPORTED, "batch too large for one launch");
    g.wgs = (int)start;
    put(host, g, kv.second);
    b.fft_groups.push_back(g);
  }
  // Gram: grouped by chain and ceil(L / 16)
  std::map<std::pair<int, int>, std::vector<GramItem>> gram;
  for (auto& s : b.pb) {
    const Plan& p = *s.plan;
    GramItem it{};
    it.qhat = ws + s.ws_qhat;
    it.sqrtw = c128(b) ? (const void*)p.d_sqrtw : (const void*)p.d_sqrtw32;
    it.part = reinterpret_cast<double*>(ws + s.ws_part);
    it.M = p.M;
    it.ldq = s.ldq;
    it.L = (int)p.nblocks;
    it.S = p.gram_split;
    it.K = (int)p.nfreq;
    const bool aligned = ((uintptr_t)it.qhat % 16 == 0) && ((uintptr_t)it.sqrtw % 16 == 0);
    it.vec = aligned && (c128(b) || s.ldq % 2 == 0);
    gram[{chain_of(p), p.gram_dim / 16}].push_back(it);
  }
  b.gram_groups.clear();
  for (auto& kv : gram) {
    Group g;
    g.chain = kv.first.first;
    g.key = kv.first.second;
    // the longest slices first (as for the transform)
    std::stable_sort(kv.second.begin(), kv.second.end(), [](const GramItem& x, const GramItem& y) {
      return (x.M + x.S - 1) / x.S > (y.M + y.S - 1) / y.S;
    });
    int64_t start = 0;
    for (auto& it : kv.second) {
      it.start = (int)start;
      start += gram_group_wgs(g.key, it.S, it.K);
    }
    if (start > 0x7fffffff) return fail(SPOD_ERR_UNSUPPORTED, "batch too large for one launch");
    g.wgs = (int)start;
    put(host, g, kv.second);
    b.gram_groups.push_back(g);
  }
  // combine, modes: one group per chain; eigensolve: by chain and L bucket
  std::vector<CombineItem> cb[NCHAIN];
  std::map<std::pair<int, int>, std::vector<EigItem>> eg;
  std::map<std::pair<int, int>, int64_t> s_eg;
  std::vector<ModesItem> md[NCHAIN];
  int64_t s_cb[NCHAIN] = {}, s_md[NCHAIN] = {};
  b.modes_lds = 0;
  for (auto& s : b.pb) {
    const Plan& p = *s.plan;
    const size_t D = (size_t)p.gram_dim;
    const int K = (int)p.nfreq, L = (int)p.nblocks;
    const int ch = chain_of(p);
    CombineItem c{};
    c.part = ws + s.ws_part;
    c.gram = ws + s.ws_gram;
    c.L = L;
    c.D = (int)D;
    c.S = p.gram_split;
    c.start = (int)s_cb[ch];
    s_cb[ch] += K;
    cb[ch].push_back(c);
    EigItem e{};
    e.gram = ws + s.ws_gram;
    e.lam = reinterpret_cast<double*>(out + s.o_lam);
    e.psi = out + s.o_psi;
    e.info = reinterpret_cast<int32_t*>(out + s.o_info);
    e.L = L;
    const std::pair<int, int> lb{ch, L <= 16 ? 16 : (L <= 32 ? 32 : 64)};
    e.start = (int)s_eg[lb];
    s_eg[lb] += K;
    eg[lb].push_back(e);
    ModesItem m{};
    m.qhat = ws + s.ws_qhat;
    m.lam = e.lam;
    m.psi = e.psi;
    m.phi = out + s.o_phi;
    m.n_valid = reinterpret_cast<int32_t*>(out + s.o_nvalid);
    m.M = p.M;
    m.ldq = s.ldq;
    m.L = L;
    m.n_modes = s.n_modes;
    // the same choice as the single-problem launch: phi rows (stride M) must
    // take whole pairs
    m.pair = !c128(b) && p.M % 2 == 0 && (uintptr_t)m.qhat % 16 == 0 && (uintptr_t)m.phi % 16 == 0;
    m.tiles = (int)(((m.pair ? p.M / 2 : p.M) + 255) / 256);
    m.eps = c128(b) ? 1e-12 : 1e-6;
    m.start = (int)s_md[ch];
    s_md[ch] += (int64_t)K * m.tiles;
    md[ch].push_back(m);
    b.modes_lds = std::max(b.modes_lds, csize(b) * (size_t)L * (size_t)s.n_modes);
  }
  for (int ch = 0; ch < NCHAIN; ++ch) {
    if (s_md[ch] > 0x7fffffff) return fail(SPOD_ERR_UNSUPPORTED, "batch too large for one launch");
    b.comb_g[ch] = Group{};
    b.comb_g[ch].chain = ch;
    put(host, b.comb_g[ch], cb[ch]);
    b.comb_g[ch].wgs = (int)s_cb[ch];
    b.modes_g[ch] = Group{};
    b.modes_g[ch].chain = ch;
    put(host, b.modes_g[ch], md[ch]);
    b.modes_g[ch].wgs = (int)s_md[ch];
  }
  b.eig_groups.clear();
  for (auto& kv : eg) {
    Group g;
    g.chain = kv.first.first;
    g.key = kv.first.second;
    put(host, g, kv.second);
    g.wgs = (int)s_eg[kv.first];
    b.eig_groups.push_back(g);
  }

  // one work-queue counter per grouped launch
  int nq = 0;
  for (auto* gs : {&b.fft_groups, &b.gram_groups, &b.eig_groups})
    for (Group& g : *gs) g.queue = nq++;
  for (int ch = 0; ch < NCHAIN; ++ch) b.modes_g[ch].queue = nq++;
  if (nq > NQUEUE) return fail(SPOD_ERR_UNSUPPORTED, "too many grouped launches");
  b.n_queue = nq;

  if (host.size() > b.table_cap) {
    if (b.d_table) (void)hipFree(b.d_table);
    b.d_table = nullptr;
    b.table_cap = 0;
    hipError_t e = hipMalloc(&b.d_table, host.size());
    if (e != hipSuccess) return e == hipErrorOutOfMemory ? fail(SPOD_ERR_ALLOC, "batch tables")
                                                         : hip_fail(e, "hipMalloc");
    b.table_cap = host.size();
  }
  hipError_t e = hipMemcpy(b.d_table, host.data(), host.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  return SPOD_OK;
}

template <typename It>
const It* at(const Batch& b, const Group& g) {
  return reinterpret_cast<const It*>(static_cast<const char*>(b.d_table) + g.off);
}

// Enqueue the whole forward pass on `st`.
spod_status record(Batch& b, const void* const* q, spod_dtype dtype, char* out, char* ws,
                   hipStream_t st) {
  spod_status r = SPOD_OK;
  if (!b.grouped) {
    for (size_t i = 0; i < b.pb.size() && r == SPOD_OK; ++i) {
      const ProblemSlots& s = b.pb[i];
      const Plan& p = *s.plan;
      void* qh = ws + s.ws_qhat;
      double* lam = reinterpret_cast<double*>(out + s.o_lam);
      r = launch_blocks_fft(p, q[i], dtype, qh, reinterpret_cast<double*>(out + s.o_mean), nullptr,
                            st);
      if (r == SPOD_OK) r = launch_csd(p, qh, ws + s.ws_gram, ws + s.ws_part, st);
      if (r == SPOD_OK)
        r = launch_eig(p, ws + s.ws_gram, lam, out + s.o_psi,
                       reinterpret_cast<int32_t*>(out + s.o_info), nullptr, st);
      if (r == SPOD_OK)
        r = launch_modes(p, qh, lam, out + s.o_psi, s.n_modes, out + s.o_phi,
                         reinterpret_cast<int32_t*>(out + s.o_nvalid), nullptr, st);
    }
    return r;
  }
  for (int i : b.fft_fallback) {
    const ProblemSlots& s = b.pb[i];
    r = launch_blocks_fft(*s.plan, q[i], dtype, ws + s.ws_qhat,
                          reinterpret_cast<double*>(out + s.o_mean), nullptr, st);
    if (r != SPOD_OK) return r;
  }
  // Chain 1 (L > 32) is forked onto the side stream after the per-problem
  // transforms and joined at the end; nothing is forked when one chain is
  // empty.  (Running chain 1's transforms alone before the fork was measured
  // slower.)
  const bool two = b.modes_g[0].n > 0 && b.modes_g[1].n > 0;
  auto hip = [](hipError_t e, const char* what) { return e == hipSuccess ? SPOD_OK : hip_fail(e, what); };
  // persistent launches: every counter is zeroed before the fork, on `st`
  auto queue = [&](const Group& g) -> int* { return b.persistent ? b.d_queue + g.queue : nullptr; };
  if (b.persistent) {
    r = launch_queue_reset(b.d_queue, b.n_queue, st);
    if (r != SPOD_OK) return r;
  }
  auto transforms = [&](int ch, hipStream_t cs) {
    for (const Group& g : b.fft_groups) {
      if (g.chain != ch || r != SPOD_OK) continue;
      r = launch_fft_group(g.key, b.prec, dtype, 4, b.fft_tile, at<FftItem>(b, g), g.n, g.wgs,
                           queue(g), cs);
    }
  };
  auto rest = [&](int ch, hipStream_t cs) {
    for (const Group& g : b.gram_groups) {
      if (g.chain != ch || r != SPOD_OK) continue;
      r = launch_gram_group(b.prec, g.key, at<GramItem>(b, g), g.n, g.wgs, queue(g), cs);
    }
    if (r == SPOD_OK)
      r = launch_gram_combine_group(at<CombineItem>(b, b.comb_g[ch]), b.comb_g[ch].n,
                                    b.comb_g[ch].wgs, cs);
    for (const Group& g : b.eig_groups) {
      if (g.chain != ch || r != SPOD_OK) continue;
      r = launch_eig_group(at<EigItem>(b, g), g.n, g.wgs, b.pb[0].plan->max_sweeps, g.key,
                           b.eig_threads, queue(g), cs);
    }
    if (r == SPOD_OK)
      r = launch_modes_group(c128(b), at<ModesItem>(b, b.modes_g[ch]), b.modes_g[ch].n,
                             b.modes_g[ch].wgs, b.modes_lds, queue(b.modes_g[ch]), cs);
  };
  if (!two) {
    const int ch = b.modes_g[1].n > 0 ? 1 : 0;
    transforms(ch, st);
    rest(ch, st);
    return r;
  }
  r = hip(hipEventRecord(b.fork, st), "hipEventRecord");
  if (r == SPOD_OK) r = hip(hipStreamWaitEvent(b.side, b.fork, 0), "hipStreamWaitEvent");
  if (r != SPOD_OK) return r;
  transforms(0, st);
  rest(0, st);
  transforms(1, b.side);
  rest(1, b.side);
  // the join is recorded whatever happened, so a capture always ends whole
  spod_status rj = hip(hipEventRecord(b.join, b.side), "hipEventRecord");
  if (rj == SPOD_OK) rj = hip(hipStreamWaitEvent(st, b.join, 0), "hipStreamWaitEvent");
  if (r == SPOD_OK) r = rj;
  return r;
}

spod_status prepare(Batch& b, const void* const* q, spod_dtype dtype, void* out, void* ws) {
  bool same = b.tables_ok && out == b.out_built && ws == b.ws_built && dtype == b.dtype_built &&
              b.target_built == b.gram_target && b.tile_built == b.fft_tile;
  for (size_t i = 0; same && i < b.pb.size(); ++i) same = q[i] == b.q_built[i];
  if (same) return SPOD_OK;
  drop_graph(b);
  b.tables_ok = false;
  apply_target(b);
  spod_status r = build_tables(b, q, dtype, static_cast<char*>(out), static_cast<char*>(ws));
  if (r != SPOD_OK) return r;
  b.q_built.assign(q, q + b.pb.size());
  b.out_built = out;
  b.ws_built = ws;
  b.dtype_built = dtype;
  b.target_built = b.gram_target;
  b.tile_built = b.fft_tile;
  b.tables_ok = true;
  return SPOD_OK;
}

spod_status run(Batch& b, const void* const* q, spod_dtype dtype, void* out, void* ws,
                hipStream_t st, bool graph) {
  spod_status r = prepare(b, q, dtype, out, ws);
  if (r != SPOD_OK) return r;
  char* o = static_cast<char*>(out);
  char* w = static_cast<char*>(ws);
  if (!graph) return record(b, q, dtype, o, w, st);
  if (!b.exec) {
    hipError_t e = hipStreamBeginCapture(b.cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    r = record(b, q, dtype, o, w, b.cap_stream);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b.cap_stream, &g);
    if (r != SPOD_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b.exec = nullptr;
      return hip_fail(e, "hipGraphInstantiate");
    }
  }
  hipError_t e = hipGraphLaunch(b.exec, st);
  return e == hipSuccess ? SPOD_OK : hip_fail(e, "hipGraphLaunch");
}

spod_status check_call(Batch* b, const void* const* q, spod_dtype dtype, void* out, void* ws,
                       size_t ws_bytes) {
  if (!b) return fail(SPOD_ERR_INVALID_ARG, "batch is NULL");
  if (!q || !out || !ws) return fail(SPOD_ERR_INVALID_ARG, "q, out and ws are required");
  if (dtype != SPOD_F32 && dtype != SPOD_F64) return fail(SPOD_ERR_INVALID_ARG, "dtype");
  for (size_t i = 0; i < b->pb.size(); ++i)
    if (!q[i]) return fail(SPOD_ERR_INVALID_ARG, "q[" + std::to_string(i) + "] is NULL");
  if ((uintptr_t)out % 256 || (uintptr_t)ws % 256)
    return fail(SPOD_ERR_INVALID_ARG, "out and ws must be 256-byte aligned");
  if (ws_bytes < b->ws_bytes)
    return fail(SPOD_ERR_WORKSPACE, "workspace of " + std::to_string(b->ws_bytes) + " bytes required");
  int cur = -1;
  hipError_t e = hipGetDevice(&cur);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (cur != b->device) return fail(SPOD_ERR_INVALID_ARG, "batch belongs to another device");
  if (!b->started) {
    b->started = true;
    for (auto& s : b->pb) freeze(*s.plan);
  }
  return SPOD_OK;
}

// FNV-1a over the shapes, precision and n_modes: the autotune cache key
std::string batch_key(const Batch& b) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](int64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (uint64_t)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  mix((int64_t)b.prec);
  for (auto& s : b.pb) {
    mix(s.plan->M);
    mix(s.plan->nt);
    mix(s.plan->nfft);
    mix(s.plan->noverlap);
    mix(s.n_modes);
  }
  char buf[32];
  std::snprintf(buf, sizeof buf, "%016" PRIx64, h);
  return buf;
}

// The launch shapes the autotuner chooses.
struct Shapes {
  int64_t gram_target = 0;   // 0: not found
  int fft_tile = 0, eig_threads = 0, persistent = 0;
};

int64_t json_int(const std::string& line, const char* name, int64_t dflt) {
  const std::string k = std::string("\"") + name + "\": ";
  const size_t p = line.find(k);
  return p == std::string::npos ? dflt : std::strtoll(line.c_str() + p + k.size(), nullptr, 10);
}

// The last line of the JSON-lines cache with this key.
Shapes cache_lookup(const char* path, const std::string& key) {
  std::ifstream f(path);
  std::string line;
  Shapes found;
  const std::string kk = "\"key\": \"" + key + "\"";
  while (std::getline(f, line)) {
    if (line.find(kk) == std::string::npos) continue;
    Shapes s;
    s.gram_target = json_int(line, "gram_target", 0);
    s.fft_tile = (int)json_int(line, "fft_tile", 0);
    s.eig_threads = (int)json_int(line, "eig_threads", 0);
    s.persistent = (int)json_int(line, "persistent", 0);
    const bool ok = s.gram_target >= 64 && (s.fft_tile == 0 || s.fft_tile == 16 || s.fft_tile == 32) &&
                    (s.eig_threads == 0 || s.eig_threads == 256 || s.eig_threads == 1024) &&
                    (s.persistent == 0 || s.persistent == 1);
    if (ok) found = s;
  }
  return found;
}

void set_shapes(Batch& b, const Shapes& s) {
  b.gram_target = s.gram_target;
  b.fft_tile = s.fft_tile;
  b.eig_threads = s.eig_threads;
  b.persistent = s.persistent;
}

}  // namespace
}  // namespace spod

using namespace spod;

extern "C" {

spod_status spod_batch_create(const spod_problem* problems, int64_t n, spod_precision precision,
                              int64_t n_modes, spod_batch* out) {
  return guarded([&]() -> spod_status {
    if (!out) return fail(SPOD_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!problems || n < 1) return fail(SPOD_ERR_INVALID_ARG, "need at least one problem");
    if (n > 65536) return fail(SPOD_ERR_INVALID_ARG, "at most 65536 problems");
    if (n_modes < 1) return fail(SPOD_ERR_INVALID_ARG, "n_modes must be >= 1");
    if (precision != SPOD_PREC_FP64 && precision != SPOD_PREC_FP32 &&
        precision != SPOD_PREC_BF16X4 && precision != SPOD_PREC_FP16X4)
      return fail(SPOD_ERR_INVALID_ARG, "unknown precision");
    Batch* b = new (std::nothrow) Batch();
    if (!b) return fail(SPOD_ERR_ALLOC, "batch");
    b->prec = precision;
    b->pb.resize((size_t)n);
    spod_status st = SPOD_OK;
    for (int64_t i = 0; i < n && st == SPOD_OK; ++i) {
      const spod_problem& d = problems[i];
      spod_plan h = nullptr;
      st = spod_plan_create(d.nspace, d.nvar, d.nt, d.nfft, d.noverlap, d.window, d.weights, &h);
      if (st != SPOD_OK) {
        fail(st, "problem " + std::to_string(i) + ": " + spod_last_error());
        break;
      }
      b->pb[i].plan = reinterpret_cast<Plan*>(h);
      st = spod_plan_set_precision(h, precision);
      if (b->pb[i].plan->nblocks > 64) st = fail(SPOD_ERR_UNSUPPORTED, "nblocks > 64");
      if (st == SPOD_OK && long_scratch_bytes(*b->pb[i].plan) > 0)
        st = fail(SPOD_ERR_UNSUPPORTED, "a batch takes blocks that fit one workgroup's LDS");
      b->pb[i].n_modes = (int)std::min<int64_t>(n_modes, b->pb[i].plan->nblocks);
    }
    if (st == SPOD_OK) {
      hipError_t e = hipGetDevice(&b->device);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
      if (e == hipSuccess) e = hipMalloc(&b->d_queue, sizeof(int) * NQUEUE);
      if (e != hipSuccess) st = hip_fail(e, "batch stream");
    }
    if (st != SPOD_OK) {
      const std::string msg = spod_last_error();
      spod_batch_destroy(reinterpret_cast<spod_batch>(b));
      fail(st, msg.substr(msg.find(": ") == std::string::npos ? 0 : msg.find(": ") + 2));
      return st;
    }
    apply_target(*b);
    layout(*b);
    *out = reinterpret_cast<spod_batch>(b);
    return SPOD_OK;
  });
}

spod_status spod_batch_set_option(spod_batch batch, spod_batch_option opt, int64_t value) {
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (!b) return fail(SPOD_ERR_INVALID_ARG, "batch is NULL");
  if (b->started) return fail(SPOD_ERR_INVALID_ARG, "batch already used");
  switch (opt) {
    case SPOD_BATCH_GROUPED:
      if (value != 0 && value != 1) return fail(SPOD_ERR_INVALID_ARG, "grouped is 0 or 1");
      b->grouped = value != 0;
      break;
    case SPOD_BATCH_GRAPH:
      if (value != 0 && value != 1) return fail(SPOD_ERR_INVALID_ARG, "graph is 0 or 1");
      b->use_graph = value != 0;
      break;
    case SPOD_BATCH_GRAM_TARGET:
      if (value < 64 || value > (int64_t(1) << 24))
        return fail(SPOD_ERR_INVALID_ARG, "gram target in [64, 2^24]");
      b->gram_target = value;
      apply_target(*b);
      layout(*b);
      break;
    case SPOD_BATCH_FFT_TILE:
      if (value != 0 && value != 16 && value != 32)
        return fail(SPOD_ERR_INVALID_ARG, "transform tile is 0, 16 or 32");
      b->fft_tile = (int)value;
      break;
    case SPOD_BATCH_EIG_THREADS:
      if (value != 0 && value != 256 && value != 1024)
        return fail(SPOD_ERR_INVALID_ARG, "eigensolver threads are 0, 256 or 1024");
      b->eig_threads = (int)value;
      break;
    case SPOD_BATCH_PERSISTENT:
      if (value != 0 && value != 1) return fail(SPOD_ERR_INVALID_ARG, "persistent is 0 or 1");
      b->persistent = (int)value;
      break;
    default:
      return fail(SPOD_ERR_INVALID_ARG, "unknown option");
  }
  return SPOD_OK;
}

spod_status spod_batch_get_option(spod_batch batch, spod_batch_option opt, int64_t* value) {
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (!b || !value) return fail(SPOD_ERR_INVALID_ARG, "batch and value are required");
  switch (opt) {
    case SPOD_BATCH_GROUPED: *value = b->grouped; break;
    case SPOD_BATCH_GRAPH: *value = b->use_graph; break;
    case SPOD_BATCH_GRAM_TARGET: *value = b->gram_target; break;
    case SPOD_BATCH_FFT_TILE: *value = b->fft_tile; break;
    case SPOD_BATCH_EIG_THREADS: *value = b->eig_threads; break;
    case SPOD_BATCH_PERSISTENT: *value = b->persistent; break;
    default: return fail(SPOD_ERR_INVALID_ARG, "unknown option");
  }
  return SPOD_OK;
}

spod_status spod_batch_query(spod_batch batch, size_t* workspace_bytes, size_t* output_bytes) {
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (!b) return fail(SPOD_ERR_INVALID_ARG, "batch is NULL");
  if (workspace_bytes) *workspace_bytes = b->ws_bytes;
  if (output_bytes) *output_bytes = b->out_bytes;
  return SPOD_OK;
}

spod_status spod_batch_item_info(spod_batch batch, int64_t i, spod_batch_item* item) {
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (!b) return fail(SPOD_ERR_INVALID_ARG, "batch is NULL");
  if (!item || i < 0 || i >= (int64_t)b->pb.size())
    return fail(SPOD_ERR_INVALID_ARG, "item index out of range");
  const ProblemSlots& s = b->pb[(size_t)i];
  item->M = s.plan->M;
  item->nblocks = s.plan->nblocks;
  item->nfreq = s.plan->nfreq;
  item->n_modes = s.n_modes;
  item->mean = s.o_mean;
  item->lam = s.o_lam;
  item->psi = s.o_psi;
  item->info = s.o_info;
  item->phi = s.o_phi;
  item->n_valid = s.o_nvalid;
  return SPOD_OK;
}

spod_status spod_batch_forward(spod_batch batch, const void* const* q, spod_dtype dtype,
                               void* out, void* ws, size_t ws_bytes, spod_stream stream) {
  return guarded([&]() -> spod_status {
    Batch* b = reinterpret_cast<Batch*>(batch);
    spod_status st = check_call(b, q, dtype, out, ws, ws_bytes);
    if (st != SPOD_OK) return st;
    return run(*b, q, dtype, out, ws, (hipStream_t)stream, b->use_graph);
  });
}

spod_status spod_batch_autotune(spod_batch batch, const void* const* q, spod_dtype dtype,
                                void* out, void* ws, size_t ws_bytes, spod_stream stream,
                                const char* cache_path, int64_t* chosen) {
  return guarded([&]() -> spod_status {
    Batch* b = reinterpret_cast<Batch*>(batch);
    spod_status st = check_call(b, q, dtype, out, ws, ws_bytes);
    if (st != SPOD_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    const std::string key = batch_key(*b);
    Shapes best = cache_path ? cache_lookup(cache_path, key) : Shapes{};
    if (best.gram_target <= 0) {
      hipEvent_t e0 = nullptr, e1 = nullptr;
      hipError_t e = hipEventCreate(&e0);
      if (e == hipSuccess) e = hipEventCreate(&e1);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
      std::ostringstream log;
      // one untimed pass (it builds the tables), then the best of two timed
      // passes, without a graph
      auto time_shapes = [&](const Shapes& c, float* best_ms) -> spod_status {
        set_shapes(*b, c);
        spod_status r = run(*b, q, dtype, out, ws, s, false);
        *best_ms = 0.0f;
        for (int rep = 0; rep < 2 && r == SPOD_OK; ++rep) {
          float ms = 0.0f;
          hipError_t x = hipEventRecord(e0, s);
          if (x == hipSuccess) r = run(*b, q, dtype, out, ws, s, false);
          if (r != SPOD_OK) break;
          if (x == hipSuccess) x = hipEventRecord(e1, s);
          if (x == hipSuccess) x = hipEventSynchronize(e1);
          if (x == hipSuccess) x = hipEventElapsedTime(&ms, e0, e1);
          if (x != hipSuccess) r = hip_fail(x, "autotune timing");
          if (r == SPOD_OK && (rep == 0 || ms < *best_ms)) *best_ms = ms;
        }
        return r;
      };
      // coordinate search from the defaults, one launch shape at a time:
      // the Gram split target, the transform tile, the eigensolver threads,
      // then one workgroup per unit against persistent workgroups
      Shapes cur;
      cur.gram_target = 8192;
      float cur_ms = 0.0f;
      bool have = false;
      const int64_t targets[] = {2048, 4096, 8192, 16384};
      for (int64_t t : targets) {
        Shapes c = cur;
        c.gram_target = t;
        float ms = 0.0f;
        if ((st = time_shapes(c, &ms)) != SPOD_OK) break;
        log << (have ? ", " : "") << "\"gram_target=" << t << "\": " << ms;
        if (!have || ms < cur_ms) {
          cur = c;
          cur_ms = ms;
        }
        have = true;
      }
      for (int tile : {16, 32}) {
        if (st != SPOD_OK) break;
        Shapes c = cur;
        c.fft_tile = tile;
        float ms = 0.0f;
        if ((st = time_shapes(c, &ms)) != SPOD_OK) break;
        log << ", \"fft_tile=" << tile << "\": " << ms;
        if (ms < cur_ms) {
          cur = c;
          cur_ms = ms;
        }
      }
      for (int nt : {256, 1024}) {
        if (st != SPOD_OK) break;
        Shapes c = cur;
        c.eig_threads = nt;
        float ms = 0.0f;
        if ((st = time_shapes(c, &ms)) != SPOD_OK) break;
        log << ", \"eig_threads=" << nt << "\": " << ms;
        if (ms < cur_ms) {
          cur = c;
          cur_ms = ms;
        }
      }
      if (st == SPOD_OK) {
        Shapes c = cur;
        c.persistent = 1;
        float ms = 0.0f;
        st = time_shapes(c, &ms);
        if (st == SPOD_OK) {
          log << ", \"persistent=1\": " << ms;
          if (ms < cur_ms) {
            cur = c;
            cur_ms = ms;
          }
        }
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      if (st != SPOD_OK) return st;
      best = cur;
      if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        f << "{\"key\": \"" << key << "\", \"gram_target\": " << best.gram_target
          << ", \"fft_tile\": " << best.fft_tile << ", \"eig_threads\": " << best.eig_threads
          << ", \"persistent\": " << best.persistent << ", \"ms\": {" << log.str() << "}}\n";
      }
    }
    set_shapes(*b, best);
    drop_graph(*b);
    b->tables_ok = false;
    if (chosen) *chosen = best.gram_target;
    return SPOD_OK;
  });
}

void spod_batch_destroy(spod_batch batch) {
  Batch* b = reinterpret_cast<Batch*>(batch);
  if (!b) return;
  int cur = 0;
  const bool have = hipGetDevice(&cur) == hipSuccess;
  if (have && cur != b->device) (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  drop_graph(*b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->side) (void)hipStreamDestroy(b->side);
  if (b->fork) (void)hipEventDestroy(b->fork);
  if (b->join) (void)hipEventDestroy(b->join);
  if (b->d_table) (void)hipFree(b->d_table);
  if (b->d_queue) (void)hipFree(b->d_queue);
  for (auto& s : b->pb)
    if (s.plan) spod_plan_destroy(reinterpret_cast<spod_plan>(s.plan));
  if (have && cur != b->device) (void)hipSetDevice(cur);
  delete b;
}

}  // extern "C"
