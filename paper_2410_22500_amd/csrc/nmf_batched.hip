// hsn_subspace_nmf_batched: many decompositions of eq. (4) of uneven size
// (rays x bins x K) in one stream of launches.
//
// Every phase of an iteration is one launch over the blocks of all
// instances: the float32 pass (MU, or N_V / N_D for an ANLS round), the
// row solves of an ANLS round, and the D update.  Each instance owns a range
// of blocks in each launch, its descriptor (operands, workspace, ranges) and
// its control block, so its stop test is its own: once it has converged its
// blocks return at once.  Iteration chunks (check_every MU iterations, or a
// few ANLS rounds) are captured once into hipGraphs and replayed; the step
// index comes from the instance's iter_base, advanced on the device at the
// end of each chunk, so one graph serves every replay.  The plan (descriptors,
// workspace, graphs, tuned partition) is cached in the context per batch
// shape.
//
// Kernels are compiled per K (and per bin class for the pass), since a
// kernel that picked K at run time would carry the register footprint of the
// largest K for every instance: instances are ordered by (K, bins > 1024) and
// the pass and the row solves take one launch per such group; the D update
// (modest registers) takes one launch for all.
//
// Partition: without autotuning each instance gets the workgroup count the
// single-instance call would use, so results are bitwise those of
// hsn_subspace_nmf.  The autotuner times candidate budgets of row tiles per
// workgroup (fewer, longer workgroups cut the per-workgroup N_D partials that
// the update must read, which dominate small instances) on a side copy of
// the state and keeps the fastest.
#include "nmf_common.hpp"

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace hsn {

size_t batched_update_lds(int max_k, int rule);
hipError_t batched_kernel_setup(size_t pass_lds, size_t upd_lds);
void launch_batched_pass(int K, int nq, int mode, bool obj, int n_blocks, hipStream_t st, const BatchInst *d,
                         int n_inst, int iter_local);
void launch_batched_init(int n_inst, int want_chol, hipStream_t st, const BatchInst *d);
void launch_batched_update(int rule, int n_blocks, size_t lds, hipStream_t st, const BatchInst *d, int n_inst,
                           int iter_local, bool has_obj, bool next_chol, bool bf16);
bool launch_batched_pass_bf16(int K, int nw, bool obj, int n_blocks, hipStream_t st, const BatchInst *d, int n_inst,
                              int iter_local);
int bf16_k_steps_class(int64_t ldb);
int pass_bf16_wgs(hsn_ctx *ctx, int64_t n_p);
size_t bf16_image_elems(int64_t ldb);
int64_t bf16_image_ldb(int64_t ldb);
void launch_batched_rows(int K, int n_blocks, hipStream_t st, const BatchInst *d, int n_inst, int iter_local);
void launch_batched_advance(int n_inst, int steps, hipStream_t st, const BatchInst *d);
int update_d_blocks(int n_k);

namespace {

constexpr int kRowsPerTile = 8;  // rows per tile of the float32 pass
constexpr int kPolishChunk = 4;  // ANLS rounds per replayed chunk

__global__ void set_limit_kernel(const BatchInst *__restrict__ d, int n, int limit) {
  const int i = int(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) d[i].ctrl->stop_at = limit;
}

constexpr int kBf16Rows = 16;  // rows per tile of the bfloat16 pass

struct Shape {
  int64_t n_p, n_k, ldp;
  int k;
  int64_t ldb;  // bfloat16 p pitch (bfloat16 bulk), else 0
  int nw;       // k-step class of the bfloat16 pass (1, 2, 4, 8), else 0
};

struct Group {
  int K, nq, i0, i1;  // instances [i0, i1) of the plan order
  int n_wg, n_rb;     // blocks of the group's pass / row-solve launches
  int nw = 0;         // bfloat16 groups: k-step class
};

// The instances a chunk launches: all of them, or after some have stopped
// the compacted list of the rest (so that no launch dispatches workgroups
// that would only return).
struct View {
  std::string key;           // "all" or the active set
  std::vector<Group> groups;
  std::vector<Group> groups16;  // (K, k-step class) groups of the bfloat16 pass
  int n = 0, total_ub = 0;
  BatchInst *d = nullptr;
};

struct Plan : Owned {
  std::string sig;
  int n = 0;
  std::vector<int> order;   // plan position -> problem index
  std::vector<Group> groups;
  std::vector<Group> groups16;    // bfloat16 bulk: (K, k-step class) groups
  bool bf16 = false;
  std::vector<int> wgb;           // bfloat16 pass workgroups per instance (chosen)
  int max_k = 1;
  bool need_nv = false;
  std::vector<Shape> shapes;
  std::vector<int> wg;            // pass workgroups per instance (chosen)
  std::vector<int> wg_cap;        // largest candidate (sizes the partials)
  std::vector<BatchInst> h;       // host copy of the descriptors
  BatchInst *d = nullptr;         // device descriptors
  BatchInst *d_tune = nullptr;    // descriptors of the tuning copy
  NmfCtrl *ctrl = nullptr;        // [n] contiguous (one read per chunk)
  char *mem = nullptr;            // per-instance workspace
  size_t mem_bytes = 0;
  int total_ub = 0;
  size_t upd_lds_mu = 0, upd_lds_nv = 0;
  int hist_cap = 0;
  std::vector<size_t> hist_off;
  // captured chunks: key = (kind, steps, flags)
  struct G {
    std::string view;
    int kind, steps, obj_last, chol_last;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  };
  std::vector<G> graphs;
  std::string tune_note;
  ~Plan() override {
    for (auto &g : graphs) {
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    if (mem) (void)hipFree(mem);
  }
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// ---------------------------------------------------------------------------
// On-disk cache of tuned partitions (HSN_TUNE_CACHE names the file; unset:
// no cache).  A JSON object with one entry per line,
//   "<device>|<plan signature>": {"budget_index": b, "bf16_tiles_index": t},
// read when a tuned plan is built and rewritten with the new entry after
// tuning.
// ---------------------------------------------------------------------------
std::string device_key(const hsn_ctx *ctx) {
  hipDeviceProp_t p;
  std::string arch = "gpu";
  if (hipGetDeviceProperties(&p, ctx->device) == hipSuccess) arch = p.gcnArchName;
  else (void)hipGetLastError();
  return arch + ":" + std::to_string(ctx->num_cu) + "cu";
}

const char *tune_cache_path() {
  const char *p = std::getenv("HSN_TUNE_CACHE");
  return (p && *p) ? p : nullptr;
}

struct TuneEntry {
  std::string key;
  int budget, tiles;
};

std::vector<TuneEntry> tune_cache_read() {
  std::vector<TuneEntry> out;
  const char *path = tune_cache_path();
  if (!path) return out;
  FILE *f = std::fopen(path, "r");
  if (!f) return out;
  char line[8192];
  while (std::fgets(line, sizeof(line), f)) {
    const char *q0 = std::strchr(line, '"');
    if (!q0) continue;
    const char *q1 = std::strchr(q0 + 1, '"');
    if (!q1) continue;
    const char *b = std::strstr(q1, "\"budget_index\":");
    const char *t = std::strstr(q1, "\"bf16_tiles_index\":");
    int bv = -1, tv = -1;
    if (!b || !t || std::sscanf(b + 15, "%d", &bv) != 1 || std::sscanf(t + 19, "%d", &tv) != 1) continue;
    out.push_back({std::string(q0 + 1, q1), bv, tv});
  }
  std::fclose(f);
  return out;
}

bool tune_cache_lookup(const std::string &key, int &budget, int &tiles) {
  for (const TuneEntry &e : tune_cache_read())
    if (e.key == key) {
      budget = e.budget;
      tiles = e.tiles;
      return true;
    }
  return false;
}

void tune_cache_store(const std::string &key, int budget, int tiles) {
  const char *path = tune_cache_path();
  if (!path) return;
  std::vector<TuneEntry> ent = tune_cache_read();
  bool found = false;
  for (TuneEntry &e : ent)
    if (e.key == key) {
      e.budget = budget;
      e.tiles = tiles;
      found = true;
    }
  if (!found) ent.push_back({key, budget, tiles});
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  std::fprintf(f, "{\n");
  for (size_t i = 0; i < ent.size(); ++i)
    std::fprintf(f, "\"%s\": {\"budget_index\": %d, \"bf16_tiles_index\": %d}%s\n", ent[i].key.c_str(),
                 ent[i].budget, ent[i].tiles, i + 1 < ent.size() ? "," : "");
  std::fprintf(f, "}\n");
  std::fclose(f);
  std::rename(tmp.c_str(), path);
}

// Lays out descriptors (plan order) for the partition `wgs`; pass and
// row-solve block ranges count from the first instance of the group, update
// blocks from the first instance of the batch.  Fills groups' block totals.
void layout(Plan &pl, const std::vector<int> &wgs, const std::vector<int> &wgb, const hsn_nmf_problem *probs,
            double tol, std::vector<BatchInst> &out, std::vector<Group> &groups, std::vector<Group> &groups16,
            int &tot_ub, int num_cu) {
  out.assign(pl.n, BatchInst{});
  groups = pl.groups;
  groups16 = pl.groups16;
  tot_ub = 0;
  for (Group &g : groups) {
    g.n_wg = g.n_rb = 0;
    for (int i = g.i0; i < g.i1; ++i) {
      const int q = pl.order[i];
      const Shape &s = pl.shapes[i];
      BatchInst &b = out[i];
      b.P = probs ? probs[q].p : nullptr;
      b.ldp = s.ldp;
      b.n_p = s.n_p;
      b.n_k = int(s.n_k);
      b.K = s.k;
      b.nq = s.n_k > 1024 ? 2 : 1;
      b.V = probs ? probs[q].V : nullptr;
      b.D = probs ? probs[q].D : nullptr;
      b.f_ref = (probs && probs[q].f_ref > 0.0) ? probs[q].f_ref : 0.0;
      b.tol = tol;
      b.wg0 = g.n_wg;
      b.n_wg = wgs[i];
      g.n_wg += wgs[i];
      b.ub0 = tot_ub;
      b.n_ub = update_d_blocks(int(s.n_k));
      tot_ub += b.n_ub;
      b.rb0 = g.n_rb;
      b.n_rb = int(std::min<int64_t>((s.n_p + 255) / 256, 8 * int64_t(num_cu)));
      g.n_rb += b.n_rb;
      b.Pb = (probs && pl.bf16) ? probs[q].p_bf16 : nullptr;
      b.ldb = s.ldb;
      b.ldb_img = pl.bf16 ? bf16_image_ldb(s.ldb) : 0;
    }
  }
  for (Group &g : groups16) {
    g.n_wg = 0;
    for (int i = g.i0; i < g.i1; ++i) {
      out[i].wg0b = g.n_wg;
      out[i].n_wgb = wgb[i];
      g.n_wg += wgb[i];
    }
  }
}

// Byte offsets of instance i's arrays inside the plan memory (region A).
struct InstMem {
  size_t gd, chol, part_nd, part_gv, part_obj, part_gd, nv, hist, dcopy, img, vcopy;
};

std::vector<InstMem> mem_layout(const Plan &pl, size_t &total) {
  std::vector<InstMem> m(pl.n);
  size_t off = align256(sizeof(BatchInst) * pl.n) * 2 + align256(sizeof(NmfCtrl) * pl.n) * 2;
  for (int i = 0; i < pl.n; ++i) {
    const Shape &s = pl.shapes[i];
    const int K = s.k;
    const int nub = update_d_blocks(int(s.n_k));
    InstMem &x = m[i];
    auto take = [&](size_t bytes) {
      const size_t o = off;
      off = align256(off + bytes);
      return o;
    };
    x.gd = take(sizeof(double) * 64);
    x.chol = take(sizeof(double) * 256 * kCholStride);
    x.part_nd = take(sizeof(float) * size_t(pl.wg_cap[i]) * s.n_k * K);
    x.part_gv = take(sizeof(double) * size_t(pl.wg_cap[i]) * K * K);
    x.part_obj = take(sizeof(double) * size_t(pl.wg_cap[i]));
    x.part_gd = take(sizeof(double) * size_t(nub) * K * K);
    x.nv = pl.need_nv ? take(sizeof(float) * size_t(s.n_p) * K) : 0;
    x.hist = take(sizeof(double) * size_t(pl.hist_cap));
    x.dcopy = take(sizeof(float) * size_t(s.n_k) * K);  // tuning: scratch D
    x.img = pl.bf16 ? take(sizeof(uint16_t) * bf16_image_elems(s.ldb)) : 0;
    x.vcopy = take(sizeof(float) * size_t(s.n_p) * K);  // tuning: scratch V (passes and row solves write V)
  }
  total = off + 256;
  return m;
}

// Candidate partitions.  budget <= 0: the single-instance partition
// (min(tiles, 2 x CUs) workgroups each).  Otherwise `budget` workgroups in
// all, shared in proportion to each instance's elements (at least 1, at most
// its tile count and 2 x CUs): fewer workgroups per instance mean fewer N_D
// partials for the D update to reduce.
std::vector<int> partition(const Plan &pl, int budget, int num_cu) {
  std::vector<int> w(pl.n);
  double tot = 0.0;
  for (const Shape &s : pl.shapes) tot += double(s.n_p) * double(s.n_k);
  for (int i = 0; i < pl.n; ++i) {
    const int64_t tiles = (pl.shapes[i].n_p + kRowsPerTile - 1) / kRowsPerTile;
    const int64_t cap = std::min<int64_t>(tiles, 2 * int64_t(num_cu));
    if (budget <= 0) {
      w[i] = int(cap);
    } else {
      const double share = double(budget) * double(pl.shapes[i].n_p) * double(pl.shapes[i].n_k) / tot;
      w[i] = int(std::max<int64_t>(1, std::min<int64_t>(int64_t(share + 0.5), cap)));
    }
  }
  return w;
}

void fill_pointers(Plan &pl, const std::vector<InstMem> &m, std::vector<BatchInst> &v, NmfCtrl *ctrl, bool tune) {
  for (int i = 0; i < pl.n; ++i) {
    BatchInst &b = v[i];
    b.gd = reinterpret_cast<double *>(pl.mem + m[i].gd);
    b.chol = reinterpret_cast<double *>(pl.mem + m[i].chol);
    b.part_nd = reinterpret_cast<float *>(pl.mem + m[i].part_nd);
    b.part_gv = reinterpret_cast<double *>(pl.mem + m[i].part_gv);
    b.part_obj = reinterpret_cast<double *>(pl.mem + m[i].part_obj);
    b.part_gd = reinterpret_cast<double *>(pl.mem + m[i].part_gd);
    b.NV = pl.need_nv ? reinterpret_cast<float *>(pl.mem + m[i].nv) : nullptr;
    b.hist = reinterpret_cast<double *>(pl.mem + m[i].hist);
    b.ctrl = ctrl + i;
    b.img = pl.bf16 ? reinterpret_cast<uint16_t *>(pl.mem + m[i].img) : nullptr;
    if (tune) {
      b.D = reinterpret_cast<float *>(pl.mem + m[i].dcopy);
      b.V = reinterpret_cast<float *>(pl.mem + m[i].vcopy);
      b.f_ref = 0.0;
    }
  }
}

// One pass launch per (K, bin class) group.
void pass_groups(const std::vector<Group> &gs, int mode, bool obj, hipStream_t st, const BatchInst *d, int s) {
  for (const Group &g : gs) launch_batched_pass(g.K, g.nq, mode, obj, g.n_wg, st, d + g.i0, g.i1 - g.i0, s);
}

// One bfloat16 MU pass launch per (K, k-step class) group.
void pass_groups16(const std::vector<Group> &gs, bool obj, hipStream_t st, const BatchInst *d, int s) {
  for (const Group &g : gs) launch_batched_pass_bf16(g.K, g.nw, obj, g.n_wg, st, d + g.i0, g.i1 - g.i0, s);
}

// One row-solve launch per group (its kernel is compiled for the group's K).
void rows_groups(const std::vector<Group> &gs, hipStream_t st, const BatchInst *d, int s) {
  for (const Group &g : gs) launch_batched_rows(g.K, g.n_rb, st, d + g.i0, g.i1 - g.i0, s);
}

// Queues one chunk of `steps` steps of one kind over the instances of v.
//   kind 0: MU iterations (objective and G_D factors on the last if asked)
//   kind 1: ANLS rounds
void queue_chunk(const Plan &pl, const View &v, hipStream_t st, int kind, int steps, bool obj_last, bool chol_last) {
  for (int s = 0; s < steps; ++s) {
    const bool last = s + 1 == steps;
    if (kind == 0) {
      if (pl.bf16)
        pass_groups16(v.groups16, obj_last && last, st, v.d, s);
      else
        pass_groups(v.groups, kModeMU, obj_last && last, st, v.d, s);
      launch_batched_update(kModeMU, v.total_ub, pl.upd_lds_mu, st, v.d, v.n, s, obj_last && last,
                            chol_last && last, pl.bf16);
    } else {
      pass_groups(v.groups, kModeNV, false, st, v.d, s);
      rows_groups(v.groups, st, v.d, s);
      pass_groups(v.groups, kModeND, true, st, v.d, s);
      launch_batched_update(kModeNV, v.total_ub, pl.upd_lds_nv, st, v.d, v.n, s, true, true, false);
    }
  }
  launch_batched_advance(v.n, steps, st, v.d);
}

// The still-active instances (plan order) as a compacted view in dst.
void compact(const Plan &pl, const std::vector<char> &act, BatchInst *dst, std::vector<BatchInst> &h, View &v) {
  h.clear();
  v.groups.clear();
  v.groups16.clear();
  v.key.assign(act.begin(), act.end());
  v.total_ub = 0;
  for (int j = 0; j < pl.n; ++j) {
    if (!act[j]) continue;
    BatchInst b = pl.h[j];
    const int i = int(h.size());
    if (v.groups.empty() || v.groups.back().K != b.K || v.groups.back().nq != b.nq)
      v.groups.push_back({b.K, b.nq, i, i, 0, 0});
    Group &g = v.groups.back();
    g.i1 = i + 1;
    b.wg0 = g.n_wg;
    g.n_wg += b.n_wg;
    b.rb0 = g.n_rb;
    g.n_rb += b.n_rb;
    b.ub0 = v.total_ub;
    v.total_ub += b.n_ub;
    if (pl.bf16) {
      const int nw = pl.shapes[j].nw;
      if (v.groups16.empty() || v.groups16.back().K != b.K || v.groups16.back().nw != nw) {
        Group g16{b.K, b.nq, i, i, 0, 0};
        g16.nw = nw;
        v.groups16.push_back(g16);
      }
      Group &gb = v.groups16.back();
      gb.i1 = i + 1;
      b.wg0b = gb.n_wg;
      gb.n_wg += b.n_wgb;
    }
    h.push_back(b);
  }
  v.n = int(h.size());
  v.d = dst;
}

hsn_status run_chunk(hsn_ctx *ctx, Plan &pl, const View &v, hipStream_t st, int kind, int steps, bool obj_last,
                     bool chol_last, bool use_graph) {
  if (!use_graph) {
    queue_chunk(pl, v, st, kind, steps, obj_last, chol_last);
    HSN_LAUNCHED(ctx);
    return HSN_OK;
  }
  for (auto &g : pl.graphs)
    if (g.view == v.key && g.kind == kind && g.steps == steps && g.obj_last == obj_last && g.chol_last == chol_last) {
      HSN_HIP(ctx, hipGraphLaunch(g.exec, st));
      return HSN_OK;
    }
  Plan::G g;
  g.view = v.key;
  g.kind = kind;
  g.steps = steps;
  g.obj_last = obj_last;
  g.chol_last = chol_last;
  // Captured on the context's own stream (the caller's may be the null
  // stream, which cannot capture), launched on the caller's.
  if (!ctx->cap_stream) HSN_HIP(ctx, hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
  hipStream_t cs = ctx->cap_stream;
  HSN_HIP(ctx, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  queue_chunk(pl, v, cs, kind, steps, obj_last, chol_last);
  const hipError_t le = hipGetLastError();
  const hipError_t ce = hipStreamEndCapture(cs, &g.graph);
  if (le != hipSuccess || ce != hipSuccess) {
    if (g.graph) (void)hipGraphDestroy(g.graph);
    return fail(ctx, HSN_ERR_DEVICE, "batched nmf: graph capture failed: %s",
                hipGetErrorString(le != hipSuccess ? le : ce));
  }
  if (hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipGraphDestroy(g.graph);
    return fail(ctx, HSN_ERR_DEVICE, "batched nmf: graph instantiation failed");
  }
  pl.graphs.push_back(g);
  HSN_HIP(ctx, hipGraphLaunch(g.exec, st));
  return HSN_OK;
}

}  // namespace
}  // namespace hsn

extern "C" hsn_status hsn_subspace_nmf_batched(hsn_ctx *ctx, int n, const hsn_nmf_problem *probs,
                                               const hsn_nmf_opts *o, int flags, hsn_nmf_stats *stats, void *stream) {
  using namespace hsn;
  if (!ctx) return HSN_ERR_INVALID_ARG;
  if (n < 1 || n > 4096 || !probs) return fail(ctx, HSN_ERR_INVALID_ARG, "batched nmf: need 1 <= n <= 4096 problems");
  if (!o) return fail(ctx, HSN_ERR_INVALID_ARG, "batched nmf: opts is NULL");
  if (o->algo != HSN_ALGO_MU || (o->precision != HSN_PREC_FP32 && o->precision != HSN_PREC_BF16) ||
      o->init != HSN_INIT_USER || (o->polish_rounds > 0 && o->polish_algo != HSN_ALGO_ANLS) ||
      o->polish_bf16_rounds > 0)
    return fail(ctx, HSN_ERR_UNSUPPORTED,
                "batched nmf: MU bulk (float32 or bfloat16) + float32 ANLS polish from a user start only");
  const bool bf16 = o->precision == HSN_PREC_BF16 && o->max_iter > 0;
  if (o->max_iter < 0 || o->check_every < 1 || o->polish_rounds < 0)
    return fail(ctx, HSN_ERR_INVALID_ARG, "batched nmf: max_iter >= 0, check_every >= 1, polish_rounds >= 0 required");
  if (flags & ~(HSN_BATCH_GRAPH | HSN_BATCH_AUTOTUNE)) return fail(ctx, HSN_ERR_INVALID_ARG, "batched nmf: bad flags");
  for (int i = 0; i < n; ++i) {
    const hsn_nmf_problem &q = probs[i];
    if (q.k < 1 || q.k > 8) return fail(ctx, HSN_ERR_SHAPE, "batched nmf: problem %d: k must be in 1..8", i);
    if (q.n_p < 1 || q.n_k < 1 || q.n_k > 2048)
      return fail(ctx, HSN_ERR_SHAPE, "batched nmf: problem %d: need n_p >= 1 and 1 <= n_k <= 2048", i);
    if (!q.p || !q.V || !q.D) return fail(ctx, HSN_ERR_INVALID_ARG, "batched nmf: problem %d: NULL pointer", i);
    if (q.ldp < q.n_k || q.ldp % 4 != 0 || reinterpret_cast<uintptr_t>(q.p) % 16 != 0)
      return fail(ctx, HSN_ERR_INVALID_ARG, "batched nmf: problem %d: ldp >= n_k, ldp %% 4 == 0, 16-byte aligned p", i);
    if (bf16 && (!q.p_bf16 || q.ldb < q.n_k || q.ldb % 32 != 0 || q.ldb > 2048 ||
                 reinterpret_cast<uintptr_t>(q.p_bf16) % 16 != 0))
      return fail(ctx, HSN_ERR_INVALID_ARG,
                  "batched nmf: problem %d: the bfloat16 bulk needs p_bf16 (16-byte aligned) with n_k <= ldb <= 2048, "
                  "ldb %% 32 == 0", i);
    if (stats && stats[i].history_cap > 0 && !stats[i].history)
      return fail(ctx, HSN_ERR_INVALID_ARG, "batched nmf: stats[%d].history is NULL", i);
  }
  DeviceGuard dg(ctx->device);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool use_graph = flags & HSN_BATCH_GRAPH;
  const bool tune = flags & HSN_BATCH_AUTOTUNE;
  const int hist_cap = o->max_iter / o->check_every + 2 + o->polish_rounds;
  const bool need_nv = o->polish_rounds > 0;

  // Plan lookup: batch shape + schedule sizes + flags.
  std::string sig = "n=" + std::to_string(n) + ";h=" + std::to_string(hist_cap) + ";nv=" + std::to_string(need_nv) +
                    ";t=" + std::to_string(tune) + ";b=" + std::to_string(bf16);
  for (int i = 0; i < n; ++i)
    sig += ";" + std::to_string(probs[i].n_p) + "," + std::to_string(probs[i].n_k) + "," +
           std::to_string(probs[i].ldp) + "," + std::to_string(probs[i].k) +
           (bf16 ? "," + std::to_string(probs[i].ldb) : std::string());
  Plan *pl = nullptr;
  for (Owned *ow : ctx->plans) {
    Plan *c = dynamic_cast<Plan *>(ow);
    if (c && c->sig == sig) pl = c;
  }
  const double tol = o->rel_obj_tol;
  hsn_status rc0 = HSN_OK;
  if (!pl) {
    auto np = new Plan;
    np->sig = sig;
    np->n = n;
    np->need_nv = need_nv;
    np->hist_cap = hist_cap;
    np->bf16 = bf16;
    // plan order: by (K, bin class), stable; with the bfloat16 bulk by (K,
    // k-step class), which refines the bin class (n_k > 1024 <=> 8 k-steps per wave)
    np->order.resize(n);
    for (int i = 0; i < n; ++i) np->order[i] = i;
    auto nwc = [&](int i) { return bf16 ? bf16_k_steps_class(probs[i].ldb) : 0; };
    auto key = [&](int i) { return bf16 ? probs[i].k * 16 + nwc(i) : probs[i].k * 4 + (probs[i].n_k > 1024 ? 2 : 1); };
    auto key32 = [&](int i) { return probs[i].k * 4 + (probs[i].n_k > 1024 ? 2 : 1); };
    std::stable_sort(np->order.begin(), np->order.end(), [&](int a, int b) { return key(a) < key(b); });
    for (int j = 0; j < n; ++j) {
      const int i = np->order[j];
      np->shapes.push_back({probs[i].n_p, probs[i].n_k, probs[i].ldp, probs[i].k, bf16 ? probs[i].ldb : 0, nwc(i)});
      np->max_k = std::max(np->max_k, probs[i].k);
      if (np->groups.empty() || key32(np->order[np->groups.back().i0]) != key32(i))
        np->groups.push_back({probs[i].k, probs[i].n_k > 1024 ? 2 : 1, j, j + 1, 0, 0});
      else
        np->groups.back().i1 = j + 1;
      if (bf16) {
        if (np->groups16.empty() || key(np->order[np->groups16.back().i0]) != key(i)) {
          Group g{probs[i].k, probs[i].n_k > 1024 ? 2 : 1, j, j + 1, 0, 0};
          g.nw = nwc(i);
          np->groups16.push_back(g);
        } else {
          np->groups16.back().i1 = j + 1;
        }
      }
    }
    const int nc = ctx->num_cu;
    const int budgets[] = {0, 2 * nc, 4 * nc, 8 * nc, 16 * nc};
    const std::vector<int> cands[] = {partition(*np, budgets[0], nc), partition(*np, budgets[1], nc),
                                      partition(*np, budgets[2], nc), partition(*np, budgets[3], nc),
                                      partition(*np, budgets[4], nc)};
    // bfloat16 pass: at least `tiles` 16-row tiles per workgroup (1 = the
    // single-instance partition); more tiles per workgroup stage the D
    // operand image fewer times on small instances
    const int tile_cands[] = {1, 2, 4, 8};
    std::vector<int> bcands[4];
    for (int c = 0; c < 4; ++c) {
      bcands[c].assign(n, 0);
      for (int j = 0; bf16 && j < n; ++j) {
        const int64_t tiles = (np->shapes[j].n_p + kBf16Rows - 1) / kBf16Rows;
        bcands[c][j] = int(std::max<int64_t>(
            1, std::min<int64_t>(nc, (tiles + tile_cands[c] - 1) / tile_cands[c])));
      }
    }
    np->wg_cap.assign(n, 1);
    for (auto &c : cands)
      for (int i = 0; i < n; ++i) np->wg_cap[i] = std::max(np->wg_cap[i], c[i]);
    for (auto &c : bcands)
      for (int i = 0; i < n; ++i) np->wg_cap[i] = std::max(np->wg_cap[i], c[i]);
    size_t total = 0;
    const std::vector<InstMem> m = mem_layout(*np, total);
    if (hipMalloc(&np->mem, total) != hipSuccess) {
      (void)hipGetLastError();
      delete np;
      return fail(ctx, HSN_ERR_OOM, "batched nmf: cannot allocate %zu bytes of plan memory", total);
    }
    np->mem_bytes = total;
    np->d = reinterpret_cast<BatchInst *>(np->mem);
    np->d_tune = reinterpret_cast<BatchInst *>(np->mem + align256(sizeof(BatchInst) * n));
    np->ctrl = reinterpret_cast<NmfCtrl *>(np->mem + align256(sizeof(BatchInst) * n) * 2);
    NmfCtrl *tctrl = reinterpret_cast<NmfCtrl *>(np->mem + align256(sizeof(BatchInst) * n) * 2 +
                                                 align256(sizeof(NmfCtrl) * n));
    np->upd_lds_mu = batched_update_lds(np->max_k, kModeMU);
    np->upd_lds_nv = batched_update_lds(np->max_k, kModeNV);
    if (batched_kernel_setup(0, std::max(np->upd_lds_mu, np->upd_lds_nv)) != hipSuccess) {
      (void)hipGetLastError();
      delete np;
      return fail(ctx, HSN_ERR_DEVICE, "batched nmf: kernel attribute setup failed");
    }
    np->wg = cands[0];
    np->wgb = bcands[0];
    int best_c = 0, best_b = 0;
    const std::string cache_key = device_key(ctx) + "|" + sig;
    const bool cached = tune && tune_cache_lookup(cache_key, best_c, best_b) && best_c >= 0 && best_c < 5 &&
                        best_b >= 0 && best_b < 4;
    if (tune && cached) {
      np->tune_note = "cached: budget " + std::to_string(budgets[best_c]) + ", bf16 tiles per workgroup " +
                      std::to_string(tile_cands[best_b]);
    } else if (tune) {
      // Time each candidate on the tuning copy (scratch V and D, control
      // and history of their own; p only read): the float32 budgets with one
      // ANLS round (N_V pass, row solves, N_D pass, D update) when polish
      // rounds follow, else one float32 MU iteration; the bfloat16
      // partitions with one MU iteration on the matrix cores.  A candidate
      // replaces the default only when it is 3 % faster (timing noise).
      hipEvent_t e0, e1;
      HSN_HIP(ctx, hipEventCreate(&e0));
      HSN_HIP(ctx, hipEventCreate(&e1));
      auto time_candidate = [&](const std::vector<int> &wgs, const std::vector<int> &wgb, bool on_bf16,
                                float &out_ms) -> hsn_status {
        std::vector<BatchInst> v;
        std::vector<Group> tg, tg16;
        int tu;
        layout(*np, wgs, wgb, probs, 0.0, v, tg, tg16, tu, ctx->num_cu);
        fill_pointers(*np, m, v, tctrl, true);
        HSN_HIP(ctx, hipMemcpyAsync(np->d_tune, v.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice, st));
        for (int j = 0; j < n; ++j) {
          const int i = np->order[j];
          HSN_HIP(ctx, hipMemcpyAsync(v[j].D, probs[i].D, sizeof(float) * probs[i].n_k * probs[i].k,
                                      hipMemcpyDeviceToDevice, st));
          HSN_HIP(ctx, hipMemcpyAsync(v[j].V, probs[i].V, sizeof(float) * probs[i].n_p * probs[i].k,
                                      hipMemcpyDeviceToDevice, st));
        }
        launch_batched_init(n, need_nv && !on_bf16 ? 1 : 0, st, np->d_tune);
        out_ms = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
          HSN_HIP(ctx, hipEventRecord(e0, st));
          if (on_bf16) {
            pass_groups16(tg16, false, st, np->d_tune, 0);
            launch_batched_update(kModeMU, tu, np->upd_lds_mu, st, np->d_tune, n, 0, false, false, true);
          } else if (need_nv) {
            pass_groups(tg, kModeNV, false, st, np->d_tune, 0);
            rows_groups(tg, st, np->d_tune, 0);
            pass_groups(tg, kModeND, true, st, np->d_tune, 0);
            launch_batched_update(kModeNV, tu, np->upd_lds_nv, st, np->d_tune, n, 0, true, true, false);
          } else {
            pass_groups(tg, kModeMU, false, st, np->d_tune, 0);
            launch_batched_update(kModeMU, tu, np->upd_lds_mu, st, np->d_tune, n, 0, false, false, false);
          }
          HSN_HIP(ctx, hipEventRecord(e1, st));
          HSN_HIP(ctx, hipEventSynchronize(e1));
          float ms = 0.f;
          HSN_HIP(ctx, hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) out_ms += ms;
        }
        HSN_LAUNCHED(ctx);
        out_ms /= 2;
        return HSN_OK;
      };
      float best = 1e30f;
      for (int c = 0; c < 5; ++c) {
        float ms = 0.f;
        if ((rc0 = time_candidate(cands[c], bcands[0], false, ms)) != HSN_OK) {
          delete np;
          return rc0;
        }
        if (c == 0 || ms < 0.97f * best) {
          best = ms;
          best_c = c;
        }
        char buf[96];
        std::snprintf(buf, sizeof(buf), "%sbudget %d: %.3f ms", c ? "; " : "", budgets[c], ms);
        np->tune_note += buf;
      }
      np->tune_note += " -> budget " + std::to_string(budgets[best_c]);
      if (bf16) {
        best = 1e30f;
        for (int c = 0; c < 4; ++c) {
          float ms = 0.f;
          if ((rc0 = time_candidate(cands[best_c], bcands[c], true, ms)) != HSN_OK) {
            delete np;
            return rc0;
          }
          if (c == 0 || ms < 0.97f * best) {
            best = ms;
            best_b = c;
          }
          char buf[96];
          std::snprintf(buf, sizeof(buf), "; bf16 %d tiles/wg: %.3f ms", tile_cands[c], ms);
          np->tune_note += buf;
        }
        np->tune_note += " -> " + std::to_string(tile_cands[best_b]) + " tiles/wg";
      }
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      tune_cache_store(cache_key, best_c, best_b);
    }
    if (tune) {
      np->wg = cands[best_c];
      np->wgb = bcands[best_b];
    }
    layout(*np, np->wg, np->wgb, nullptr, tol, np->h, np->groups, np->groups16, np->total_ub, ctx->num_cu);
    fill_pointers(*np, m, np->h, np->ctrl, false);
    for (int i = 0; i < n; ++i) np->hist_off.push_back(m[i].hist);
    {
      int tot = 0;
      for (int w : np->wg) tot += w;
      char buf[160];
      std::snprintf(buf, sizeof(buf), "%d instances in %zu (K, bin class) groups; %d pass workgroups, %d update blocks%s",
                    n, np->groups.size(), tot, np->total_ub, tune ? "; tuning: " : "");
      np->tune_note = buf + np->tune_note;
    }
    ctx->plans.push_back(np);
    pl = np;
  }
  ctx->last_plan_note = pl->tune_note;

  // Per call: operands, stop references and tolerance into the descriptors.
  for (int j = 0; j < n; ++j) {
    const int i = pl->order[j];
    pl->h[j].P = probs[i].p;
    pl->h[j].V = probs[i].V;
    pl->h[j].D = probs[i].D;
    pl->h[j].f_ref = probs[i].f_ref > 0.0 ? probs[i].f_ref : 0.0;
    pl->h[j].tol = tol;
    pl->h[j].Pb = bf16 ? probs[i].p_bf16 : nullptr;
  }
  const int n_steps = o->max_iter + o->polish_rounds;
  const bool first_exact = o->max_iter == 0 && o->polish_rounds > 0;
  if (stats) HSN_HIP(ctx, hipEventRecord(ctx->ev0, st));
  HSN_HIP(ctx, hipMemcpyAsync(pl->d, pl->h.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice, st));
  launch_batched_init(n, first_exact ? 1 : 0, st, pl->d);
  // Steps beyond the schedule (the tail of the last polish chunk) return at once.
  set_limit_kernel<<<(n + 63) / 64, 64, 0, st>>>(pl->d, n, n_steps);
  HSN_LAUNCHED(ctx);

  bool any_ref = false;
  for (int i = 0; i < n; ++i) any_ref |= probs[i].f_ref > 0.0;
  std::vector<NmfCtrl> hc(n);
  auto all_stopped = [&](int done) -> int {  // -1 on error, 1 if every instance stopped before `done`
    if (hipMemcpyAsync(hc.data(), pl->ctrl, sizeof(NmfCtrl) * n, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return -1;
    for (int i = 0; i < n; ++i)
      if (hc[i].stop_at > done) return 0;
    return 1;
  };
  hsn_status rc = HSN_OK;
  int done = 0;
  bool stopped = false;
  const bool polish_follows = o->polish_rounds > 0;
  View full;
  full.key = "all";
  full.groups = pl->groups;
  full.groups16 = pl->groups16;
  full.n = n;
  full.total_ub = pl->total_ub;
  full.d = pl->d;
  View cur = full;
  std::vector<BatchInst> h_act;
  std::vector<char> act(n, 1);
  // After a chunk: stop when every instance has stopped, else drop the
  // stopped ones from the launches.
  auto after_chunk = [&]() -> hsn_status {
    if (!any_ref || done >= n_steps) return HSN_OK;
    const int a = all_stopped(done);
    if (a < 0) return fail(ctx, HSN_ERR_DEVICE, "batched nmf: control read failed");
    stopped = a == 1;
    if (stopped) return HSN_OK;
    bool changed = false;
    for (int j = 0; j < n; ++j) {
      const char now = hc[j].stop_at > done ? 1 : 0;
      changed |= now != act[j];
      act[j] = now;
    }
    if (changed) {
      compact(*pl, act, pl->d_tune, h_act, cur);
      HSN_HIP(ctx, hipMemcpyAsync(pl->d_tune, h_act.data(), sizeof(BatchInst) * h_act.size(), hipMemcpyHostToDevice,
                                  st));
    }
    return HSN_OK;
  };
  while (done < o->max_iter && !stopped) {
    const int c = std::min(o->check_every, o->max_iter - done);
    const bool last_bulk = done + c == o->max_iter;
    if ((rc = run_chunk(ctx, *pl, cur, st, 0, c, true, polish_follows && last_bulk, use_graph)) != HSN_OK) return rc;
    done += c;
    if ((rc = after_chunk()) != HSN_OK) return rc;
  }
  while (done < n_steps && !stopped) {
    if ((rc = run_chunk(ctx, *pl, cur, st, 1, kPolishChunk, true, true, use_graph)) != HSN_OK) return rc;
    done += kPolishChunk;
    if ((rc = after_chunk()) != HSN_OK) return rc;
  }
  if (stats) {
    HSN_HIP(ctx, hipEventRecord(ctx->ev1, st));
    HSN_HIP(ctx, hipMemcpyAsync(hc.data(), pl->ctrl, sizeof(NmfCtrl) * n, hipMemcpyDeviceToHost, st));
    HSN_HIP(ctx, hipStreamSynchronize(st));
    float ms = 0.f;
    HSN_HIP(ctx, hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    std::vector<double> h;
    for (int j = 0; j < n; ++j) {
      const int i = pl->order[j];
      hsn_nmf_stats &s = stats[i];
      const int fin = std::min(hc[j].stop_at, n_steps);
      s.ms = ms;
      s.iters = std::min(fin, o->max_iter);
      s.polish_done = std::max(0, fin - o->max_iter);
      s.polish_bf16_done = 0;
      s.fell_back = 0;
      s.history_len = 0;
      s.objective = NAN;
      const int len = std::min(hc[j].hist_len, pl->hist_cap);
      if (len > 0) {
        h.resize(len);
        HSN_HIP(ctx, hipMemcpy(h.data(), pl->mem + pl->hist_off[j], sizeof(double) * len, hipMemcpyDeviceToHost));
        s.objective = h.back();
        const int nc = std::min(len, s.history_cap);
        for (int j = 0; j < nc; ++j) s.history[j] = h[j];
        s.history_len = nc;
      }
      s.rel_obj = probs[i].f_ref > 0.0 ? (s.objective - probs[i].f_ref) / probs[i].f_ref : NAN;
    }
  }
  return HSN_OK;
}

extern "C" const char *hsn_batched_plan_info(const hsn_ctx *ctx) {
  return ctx ? ctx->last_plan_note.c_str() : "";
}
