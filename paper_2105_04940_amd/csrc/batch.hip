// Many independent block-sampling problems in one pass: the norm pass, the
// plans, the exact products and the sketched products of every problem each
// run as one launch over all problems, so a batch of small and uneven
// problems fills the chip and the whole pass can be captured as one graph.
//
// All argument tables (per-problem norm, plan and product arguments, the
// work lists of the grouped products) are built on the host when the
// batch is created or retuned and live in one device allocation owned by the
// batch; a run only launches kernels.
//
// The sketched product has two forms, both chosen among by the tuner: the
// drawn columns of M and rows of N read in place by the product (the gather
// fused into its loads), or the sketches C, D materialized first by a grouped
// gather into a workspace of the batch and then multiplied by the plain
// grouped product. The workspace holds the sketches of a group of problems
// at a time (problems taken longest first until kSketchCap bytes are used),
// so the materialized form runs one gather and one product launch per group.
// Both forms feed the matrix cores the same float32 values in the same
// order, so they give the same bits.
#include <algorithm>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "api_internal.h"

namespace {

constexpr int kProducts = 2;   // 0: exact MN, 1: sketched CD
constexpr size_t kSketchCap = size_t(32) << 30;  // bytes of materialized sketches at a time

// Bump layout over one allocation; a pass with base == nullptr measures.
struct Layout {
  char* base = nullptr;
  size_t off = 0;
  template <typename T> T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

int64_t ceil_div64(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

struct sbmm_batch_s {
  sbmm_handle h = nullptr;
  int32_t T = 0;
  std::vector<sbmm_batch_item> items;
  sbmm_batch_outputs out{};
  char* mem = nullptr;
  // device tables
  void* norm_args = nullptr;
  void* stats_args = nullptr;
  int64_t* wg_off = nullptr;
  int64_t* blk_off = nullptr;
  int64_t total_wg = 0, total_blk = 0;
  PlanLaunch* plans = nullptr;
  void* gargs[kProducts] = {};
  int32_t* item_prob[kProducts] = {};
  int32_t* item_tile[kProducts] = {};
  int64_t* part_base[kProducts] = {};
  double* part[kProducts] = {};
  float* stage = nullptr;
  const int64_t** col_end = nullptr;
  int64_t items_n[kProducts] = {}, nparts[kProducts] = {};
  // host copies used to rebuild the product tables for another configuration
  std::vector<GemmLaunch> launches[kProducts];
  std::vector<double> work_key[kProducts];   // longest-first ordering key per problem
  sbmm_batch_tuning tuning{};
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // materialized sketches (sketch configurations grouped_cfg_count() and up)
  char* sk_mem = nullptr;                 // null: only the fused form is available
  std::vector<int32_t> gm_prob;           // problems in group-major order
  std::vector<int32_t> grp_begin;         // G + 1 offsets into gm_prob
  std::vector<int64_t> grp_wg;            // gather workgroups of each group
  std::vector<int64_t> grp_items;         // G + 1 offsets into the current work list
  std::vector<GemmLaunch> mat_launch;     // per problem: the product over its materialized sketch
  void* gather_args = nullptr;            // T gather records, group-major
  int64_t* gather_wg = nullptr;           // per group its count + 1 workgroup offsets (T + G entries)
  bool exact_lds = false;                 // every exact product can take the 256 x 256 tiles
  bool sketch_lds = false;                // every product over a materialized sketch can take them
};

namespace {

sbmm_status validate_item(sbmm_handle h, int32_t t, const sbmm_batch_item& it) {
  if (it.m < 1 || it.n < 1 || it.p < 1)
    return fail(h, SBMM_E_ARG, "problem %d: shape m=%lld n=%lld p=%lld (need all >= 1)", t, (long long)it.m,
                (long long)it.n, (long long)it.p);
  if (it.n > INT32_MAX) return fail(h, SBMM_E_ARG, "problem %d: n exceeds 2^31 - 1", t);
  if (!it.M || it.ldm < it.n || !it.N || it.ldn < it.p)
    return fail(h, SBMM_E_ARG, "problem %d: M / N missing or leading dimension too small", t);
  if (!it.CD || it.ldcd < it.p || !it.MN || it.ldmn < it.p)
    return fail(h, SBMM_E_ARG, "problem %d: CD / MN missing or leading dimension too small", t);
  if (it.K < 1 || !it.block_off) return fail(h, SBMM_E_ARG, "problem %d: need K >= 1 and block offsets", t);
  if (it.block_off[0] != 0 || it.block_off[it.K] != it.n)
    return fail(h, SBMM_E_ARG, "problem %d: block offsets must start at 0 and end at n", t);
  for (int32_t k = 0; k < it.K; ++k)
    if (it.block_off[k + 1] - it.block_off[k] < 1)
      return fail(h, SBMM_E_ARG, "problem %d: block %d is empty", t, k);
  if (it.c < 1 || it.c > INT32_MAX) return fail(h, SBMM_E_ARG, "problem %d: c = %lld out of range", t, (long long)it.c);
  if (enum_raw(it.prob) != SBMM_P_UNIFORM && enum_raw(it.prob) != SBMM_P_NORM)
    return fail(h, SBMM_E_ARG, "problem %d: batches take the UNIFORM or NORM rule", t);
  return SBMM_OK;
}

int64_t max_width(const sbmm_batch_item& it) {
  int64_t w = 0;
  for (int32_t k = 0; k < it.K; ++k) w = std::max(w, it.block_off[k + 1] - it.block_off[k]);
  return w;
}

// Row splits of a problem's column-norm pass: the batch provides the
// parallelism, so a split covers up to 512 rows.
int batch_rsplit(int64_t m) { return (int)std::min<int64_t>(64, std::max<int64_t>(1, ceil_div64(m, 512))); }

int64_t tiles_for(const sbmm_batch_item& it, int cfg) {
  int64_t bm, bn;
  int w;
  grouped_cfg_shape(cfg, &bm, &bn, &w);
  return ceil_div64(it.m, bm) * ceil_div64(it.p, bn);
}

// Largest float count of the staging buffer (a tile-sized slot per work
// item) over every configuration.
size_t max_stage_floats(const std::vector<sbmm_batch_item>& items) {
  size_t best = 0;
  for (int cfg = 0; cfg < grouped_cfg_count(); ++cfg) {
    int64_t bm, bn;
    int w;
    grouped_cfg_shape(cfg, &bm, &bn, &w);
    int64_t n = 0;
    for (const auto& it : items) n += tiles_for(it, cfg);
    best = std::max(best, (size_t)n * (size_t)(bm * bn));
  }
  return best;
}

// Configurations of product g: the tile shapes, and for the sketched
// product the same shapes again over materialized sketches.
int product_cfgs(const sbmm_batch b, int g) {
  return grouped_cfg_count() * ((g == 1 && b->sk_mem) ? 2 : 1);
}

bool materialized(const sbmm_batch b, int g, int cfg) { return g == 1 && cfg >= grouped_cfg_count(); }

// Whether configuration cfg of product g can run: the LDS-direct tiles
// (tile configurations 4 and 5) take no fused gather, and need every
// problem's rows 16-byte aligned and its panels within 32-bit offsets.
bool cfg_ok(const sbmm_batch b, int g, int cfg) {
  if (cfg < 0 || cfg >= product_cfgs(b, g)) return false;
  const bool mat = materialized(b, g, cfg);
  const int tile = mat ? cfg - grouped_cfg_count() : cfg;
  if (tile != 4 && tile != 5) return true;
  if (g == 0) return b->exact_lds;
  return mat && b->sketch_lds;
}

// Rebuild and upload the tables of product g for configuration (cfg, lpt).
// Materialized sketches: the work list runs group by group (each group's
// problems in their own order), with the group boundaries kept in grp_items.
sbmm_status apply_product(sbmm_batch b, int g, int cfg, int lpt) {
  sbmm_handle h = b->h;
  const int32_t T = b->T;
  const bool mat = materialized(b, g, cfg);
  const int tcfg = mat ? cfg - grouped_cfg_count() : cfg;
  const std::vector<GemmLaunch>& src = mat ? b->mat_launch : b->launches[g];
  const size_t ab = grouped_gemm_args_bytes();
  std::vector<char> args((size_t)T * ab);
  std::vector<int64_t> base(T + 1, 0);
  for (int32_t t = 0; t < T; ++t) {
    build_grouped_gemm_args(src[t], tcfg, args.data() + (size_t)t * ab);
    base[t + 1] = base[t] + tiles_for(b->items[t], tcfg);
  }
  auto longer = [&](int32_t x, int32_t y) { return b->work_key[g][x] > b->work_key[g][y]; };
  std::vector<int32_t> order;
  if (mat) {
    b->grp_items.assign(1, 0);
    for (size_t gi = 0; gi + 1 < b->grp_begin.size(); ++gi) {
      std::vector<int32_t> part(b->gm_prob.begin() + b->grp_begin[gi], b->gm_prob.begin() + b->grp_begin[gi + 1]);
      if (lpt) std::stable_sort(part.begin(), part.end(), longer);
      else std::sort(part.begin(), part.end());
      int64_t n = 0;
      for (int32_t t : part) n += base[t + 1] - base[t];
      b->grp_items.push_back(b->grp_items.back() + n);
      order.insert(order.end(), part.begin(), part.end());
    }
  } else {
    order.resize(T);
    std::iota(order.begin(), order.end(), 0);
    if (lpt) std::stable_sort(order.begin(), order.end(), longer);
  }
  const int64_t n_items = base[T];
  std::vector<int32_t> iprob((size_t)n_items), itile((size_t)n_items);
  int64_t k = 0;
  for (int32_t t : order)
    for (int64_t l = 0; l < base[t + 1] - base[t]; ++l, ++k) {
      iprob[k] = t;
      itile[k] = (int32_t)l;
    }
  HIP_TRY(h, hipMemcpy(b->gargs[g], args.data(), args.size(), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(b->part_base[g], base.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(b->item_prob[g], iprob.data(), sizeof(int32_t) * n_items, hipMemcpyHostToDevice));
  HIP_TRY(h, hipMemcpy(b->item_tile[g], itile.data(), sizeof(int32_t) * n_items, hipMemcpyHostToDevice));
  b->items_n[g] = n_items;
  b->nparts[g] = n_items;
  b->tuning.cfg[g] = cfg;
  b->tuning.lpt[g] = lpt;
  return SBMM_OK;
}

void drop_graph(sbmm_batch b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
}

hipError_t enqueue_product(sbmm_batch b, int g, hipStream_t s) {
  GroupedLaunch L{};
  L.probs = b->gargs[g];
  L.item_prob = b->item_prob[g];
  L.item_tile = b->item_tile[g];
  L.part_base = b->part_base[g];
  L.items = b->items_n[g];
  L.nparts = b->nparts[g];
  L.stage = b->stage;
  L.cfg = b->tuning.cfg[g];
  L.gather = g == 1;
  if (!materialized(b, g, L.cfg)) return launch_grouped_gemm(L, s);
  // group by group: gather the sketches, then multiply them
  L.cfg -= grouped_cfg_count();
  L.gather = false;
  const size_t ab = batch_gather_args_bytes();
  for (size_t gi = 0; gi + 1 < b->grp_begin.size(); ++gi) {
    const int32_t first = b->grp_begin[gi], count = b->grp_begin[gi + 1] - first;
    hipError_t e = launch_batch_gather(static_cast<const char*>(b->gather_args) + (size_t)first * ab,
                                       b->gather_wg + first + gi, count, b->grp_wg[gi], s);
    if (e != hipSuccess) return e;
    GroupedLaunch G = L;
    G.item_prob = b->item_prob[g] + b->grp_items[gi];
    G.item_tile = b->item_tile[g] + b->grp_items[gi];
    G.items = b->grp_items[gi + 1] - b->grp_items[gi];
    if ((e = launch_grouped_gemm(G, s)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Place the sketches of every problem (longest expected width first) into
// groups that fit the sketch workspace, allocate it, and build the gather
// records and the products over the materialized sketches. Leaves sk_mem
// null (only the fused form) when the workspace cannot be allocated.
void setup_materialized(sbmm_batch b, const std::vector<int64_t>& lpm,
                        const std::vector<const int64_t*>& col_end, const std::vector<const int32_t*>& colmap,
                        const std::vector<const double*>& colscale) {
  const int32_t T = b->T;
  auto al = [](size_t x) { return (x + 255) & ~size_t(255); };
  std::vector<size_t> cb(T), db(T);
  size_t total = 0, most = 0;
  for (int32_t t = 0; t < T; ++t) {
    const sbmm_batch_item& it = b->items[t];
    cb[t] = al(sizeof(float) * (size_t)it.m * lpm[t]);
    db[t] = al(sizeof(float) * (size_t)lpm[t] * round_up(it.p, 4));
    total += cb[t] + db[t];
    most = std::max(most, cb[t] + db[t]);
  }
  const size_t cap = std::min(total, std::max(kSketchCap, most));
  std::vector<int32_t> order(T);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return b->work_key[1][x] > b->work_key[1][y]; });
  std::vector<size_t> at(T);
  b->grp_begin.assign(1, 0);
  size_t cur = 0;
  for (int32_t i = 0; i < T; ++i) {
    const int32_t t = order[i];
    if (cur > 0 && cur + cb[t] + db[t] > cap) {
      b->grp_begin.push_back(i);
      cur = 0;
    }
    at[t] = cur;
    cur += cb[t] + db[t];
  }
  b->grp_begin.push_back(T);
  if (hipMalloc(&b->sk_mem, cap) != hipSuccess) {
    b->sk_mem = nullptr;
    (void)hipGetLastError();   // the fused form needs no workspace
    return;
  }
  b->gm_prob = order;
  const size_t G = b->grp_begin.size() - 1;
  const size_t ab = batch_gather_args_bytes();
  std::vector<char> gargs((size_t)T * ab);
  std::vector<int64_t> wg;
  b->grp_wg.assign(G, 0);
  b->mat_launch.resize(T);
  for (size_t gi = 0; gi < G; ++gi) {
    wg.push_back(0);
    for (int32_t i = b->grp_begin[gi]; i < b->grp_begin[gi + 1]; ++i) {
      const int32_t t = order[i];
      const sbmm_batch_item& it = b->items[t];
      float* C = reinterpret_cast<float*>(b->sk_mem + at[t]);
      float* D = reinterpret_cast<float*>(b->sk_mem + at[t] + cb[t]);
      const int64_t ldd = round_up(it.p, 4);
      GatherLaunch gl{};
      gl.in_dt = SBMM_F32; gl.out_dt = SBMM_F32;
      gl.M = it.M; gl.ldm = it.ldm; gl.N = it.N; gl.ldn = it.ldn; gl.m = it.m; gl.p = it.p;
      gl.L_dev = col_end[t]; gl.L_pad_max = lpm[t]; gl.colmap = colmap[t]; gl.colscale = colscale[t];
      gl.C = C; gl.ldc = lpm[t]; gl.D = D; gl.ldd = ldd;
      wg.push_back(wg.back() + build_batch_gather_args(gl, gargs.data() + (size_t)i * ab));
      GemmLaunch mk = b->launches[1][t];
      mk.A = C; mk.lda = lpm[t]; mk.B = D; mk.ldb = ldd;
      mk.colmap = nullptr; mk.colscale = nullptr;
      b->mat_launch[t] = mk;
    }
    b->grp_wg[gi] = wg.back();
  }
  // the 256 x 256 tiles address a panel with 32-bit offsets: a sketch width
  // (C's leading dimension) past about 2^21 floats rules them out
  b->sketch_lds = true;
  for (int32_t t = 0; t < T; ++t) b->sketch_lds = b->sketch_lds && grouped_lds_ok(b->mat_launch[t]);
  hipError_t e = hipMemcpy(b->gather_args, gargs.data(), gargs.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->gather_wg, wg.data(), sizeof(int64_t) * wg.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(b->sk_mem);
    b->sk_mem = nullptr;
    (void)hipGetLastError();
  }
}

sbmm_status enqueue_pass(sbmm_batch b, hipStream_t s) {
  sbmm_handle h = b->h;
  HIP_TRY(h, launch_batch_norms(SBMM_F32, b->norm_args, b->wg_off, b->total_wg, b->stats_args, b->blk_off,
                                b->total_blk, b->T, s));
  HIP_TRY(h, launch_batch_plan(b->plans, b->T, s));
  HIP_TRY(h, enqueue_product(b, 0, s));
  HIP_TRY(h, enqueue_product(b, 1, s));
  HIP_TRY(h, launch_grouped_reduce(b->part[1], b->nparts[1], b->part_base[1], b->part[0], b->nparts[0],
                                   b->part_base[0], b->col_end, b->T, b->out.err2_mn2, b->out.L, s));
  return SBMM_OK;
}

sbmm_status check_batch(sbmm_handle h, sbmm_batch b) {
  sbmm_status st = check_handle(h);
  if (st != SBMM_OK) return st;
  if (!b) return fail(h, SBMM_E_ARG, "batch is NULL");
  if (b->h != h) return fail(h, SBMM_E_STATE, "batch belongs to another handle");
  return SBMM_OK;
}

}  // namespace

extern "C" {

sbmm_status sbmm_batch_create(sbmm_handle h, int32_t T, const sbmm_batch_item* items,
                              const sbmm_batch_outputs* out, sbmm_batch* batch) {
  sbmm_status st = check_handle(h);
  if (st != SBMM_OK) return st;
  if (!batch) return fail(h, SBMM_E_ARG, "batch is NULL");
  *batch = nullptr;
  if (T < 1 || !items) return fail(h, SBMM_E_ARG, "need T >= 1 problems");
  if (!out || !out->err2_mn2) return fail(h, SBMM_E_ARG, "outputs.err2_mn2 is required");
  for (int32_t t = 0; t < T; ++t)
    if ((st = validate_item(h, t, items[t])) != SBMM_OK) return st;

  sbmm_batch b = new (std::nothrow) sbmm_batch_s();
  if (!b) return fail(h, SBMM_E_NOMEM, "batch");
  b->h = h;
  b->T = T;
  b->items.assign(items, items + T);
  b->out = *out;

  // per-problem sizes
  std::vector<int64_t> lpm(T), rs(T);
  int64_t max_items = 0, sum_c = 0;
  for (int32_t t = 0; t < T; ++t) {
    lpm[t] = round_up(items[t].c * max_width(items[t]), SBMM_SKETCH_PAD);
    rs[t] = batch_rsplit(items[t].m);
    int64_t most = 0;
    for (int cfg = 0; cfg < grouped_cfg_count(); ++cfg) most = std::max(most, tiles_for(items[t], cfg));
    max_items += most;
    sum_c += items[t].c;
  }

  // two passes over the layout: measure, then place
  struct PerProblem {
    int64_t* off; double* partial; double* col_sq; double* row_sq; double* blk;
    uint64_t* W; uint64_t* cdf; uint64_t* Tw; int64_t* draw_off; int64_t* width; int64_t* ck;
    int32_t* idx; double* scale; int64_t* col_off; int32_t* colmap; double* colscale;
  };
  std::vector<PerProblem> pp(T);
  Layout lay;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      hipError_t e = hipMalloc(&b->mem, lay.off);
      if (e != hipSuccess) {
        b->mem = nullptr;
        delete b;
        return fail(h, SBMM_E_NOMEM, "batch tables of %zu bytes: %s", lay.off, hipGetErrorString(e));
      }
      lay = Layout{b->mem, 0};
    }
    b->norm_args = lay.take<char>((size_t)T * batch_norm_args_bytes());
    b->stats_args = lay.take<char>((size_t)T * batch_stats_args_bytes());
    b->wg_off = lay.take<int64_t>(T + 1);
    b->blk_off = lay.take<int64_t>(T + 1);
    b->plans = lay.take<PlanLaunch>(T);
    for (int g = 0; g < kProducts; ++g) {
      b->gargs[g] = lay.take<char>((size_t)T * grouped_gemm_args_bytes());
      b->item_prob[g] = lay.take<int32_t>(max_items);
      b->item_tile[g] = lay.take<int32_t>(max_items);
      b->part_base[g] = lay.take<int64_t>(T + 1);
      b->part[g] = lay.take<double>(2 * max_items);
    }
    b->stage = lay.take<float>(max_stage_floats(b->items));
    b->col_end = lay.take<const int64_t*>(T);
    b->gather_args = lay.take<char>((size_t)T * batch_gather_args_bytes());
    b->gather_wg = lay.take<int64_t>(2 * (size_t)T);
    for (int32_t t = 0; t < T; ++t) {
      const sbmm_batch_item& it = items[t];
      PerProblem& q = pp[t];
      q.off = lay.take<int64_t>(it.K + 1);
      q.partial = lay.take<double>((size_t)rs[t] * it.n);
      q.col_sq = lay.take<double>(it.n);
      q.row_sq = lay.take<double>(it.n);
      q.blk = lay.take<double>(3 * (size_t)it.K);
      q.W = lay.take<uint64_t>(it.K);
      q.cdf = lay.take<uint64_t>(it.K);
      q.Tw = lay.take<uint64_t>(1);
      q.draw_off = lay.take<int64_t>(2);
      q.width = lay.take<int64_t>(it.c);
      q.ck = lay.take<int64_t>(1);
      q.idx = out->idx ? nullptr : lay.take<int32_t>(it.c);
      q.scale = lay.take<double>(it.c);
      q.col_off = lay.take<int64_t>(it.c + 1);
      q.colmap = lay.take<int32_t>(lpm[t]);
      q.colscale = lay.take<double>(lpm[t]);
    }
  }

  // host tables
  const size_t nb = batch_norm_args_bytes(), sb = batch_stats_args_bytes();
  std::vector<char> nargs((size_t)T * nb), sargs((size_t)T * sb);
  std::vector<int64_t> wg(T + 1, 0), bo(T + 1, 0);
  std::vector<PlanLaunch> plans(T);
  std::vector<const int64_t*> col_end(T);
  std::vector<const int32_t*> colmaps(T);
  std::vector<const double*> colscales(T);
  int64_t idx_at = 0;
  for (int g = 0; g < kProducts; ++g) {
    b->launches[g].resize(T);
    b->work_key[g].resize(T);
  }
  for (int32_t t = 0; t < T; ++t) {
    const sbmm_batch_item& it = items[t];
    PerProblem& q = pp[t];
    if (out->idx) q.idx = out->idx + idx_at;
    idx_at += it.c;
    NormLaunch nl{};
    nl.dt = SBMM_F32; nl.M = it.M; nl.ldm = it.ldm; nl.N = it.N; nl.ldn = it.ldn;
    nl.m = it.m; nl.n = it.n; nl.p = it.p; nl.K = it.K; nl.off_dev = q.off;
    nl.partial = q.partial; nl.rsplit = (int)rs[t]; nl.col_sq = q.col_sq; nl.row_sq = q.row_sq; nl.blk = q.blk;
    nl.status = h->status;
    wg[t + 1] = wg[t] + build_batch_norm_args(nl, nargs.data() + (size_t)t * nb, sargs.data() + (size_t)t * sb);
    bo[t + 1] = bo[t] + it.K;

    PlanLaunch& L = plans[t];
    L = PlanLaunch{};
    L.mode = SBMM_MODE_BLOCK; L.prob = it.prob; L.alloc = SBMM_ALLOC_UNIFORM;
    L.n = it.n; L.K = it.K; L.c = it.c; L.A = it.K; L.S = 1;
    L.off_dev = q.off; L.col_sq = q.col_sq; L.row_sq = q.row_sq; L.blk = q.blk;
    L.seed = it.seed; L.trial = it.trial;
    L.W = q.W; L.cdf = q.cdf; L.T = q.Tw; L.draw_off = q.draw_off; L.width = q.width;
    L.idx = q.idx; L.scale = q.scale; L.col_off = q.col_off; L.ck = q.ck; L.p_hat = nullptr;
    L.colmap = q.colmap; L.colscale = q.colscale; L.L_pad_max = lpm[t]; L.status = h->status;
    col_end[t] = q.col_off + it.c;

    GemmLaunch ex{};
    ex.dt = SBMM_F32; ex.A = it.M; ex.lda = it.ldm; ex.B = it.N; ex.ldb = it.ldn;
    ex.m = it.m; ex.p = it.p; ex.K_host = it.n; ex.Cout = it.MN; ex.ldc = it.ldmn;
    ex.tile_part = b->part[0]; ex.stage = b->stage;
    b->launches[0][t] = ex;
    b->work_key[0][t] = (double)it.n;
    GemmLaunch sk = ex;
    sk.K_host = 0; sk.K_dev = col_end[t]; sk.Cout = it.CD; sk.ldc = it.ldcd;
    sk.Y = it.MN; sk.ldy = it.ldmn; sk.tile_part = b->part[1];
    sk.colmap = q.colmap; sk.colscale = q.colscale;
    b->launches[1][t] = sk;
    b->work_key[1][t] = (double)it.c * (double)it.n / (double)it.K;   // expected sketch width
    colmaps[t] = q.colmap;
    colscales[t] = q.colscale;
  }
  b->total_wg = wg[T];
  b->total_blk = bo[T];
  auto up = [&](void* dst, const void* src, size_t bytes) { return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice); };
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = up(b->norm_args, nargs.data(), nargs.size());
  if (e == hipSuccess) e = up(b->stats_args, sargs.data(), sargs.size());
  if (e == hipSuccess) e = up(b->wg_off, wg.data(), sizeof(int64_t) * (T + 1));
  if (e == hipSuccess) e = up(b->blk_off, bo.data(), sizeof(int64_t) * (T + 1));
  if (e == hipSuccess) e = up(b->plans, plans.data(), sizeof(PlanLaunch) * T);
  if (e == hipSuccess) e = up(b->col_end, col_end.data(), sizeof(const int64_t*) * T);
  for (int32_t t = 0; t < T && e == hipSuccess; ++t)
    e = up(pp[t].off, items[t].block_off, sizeof(int64_t) * (items[t].K + 1));
  if (e != hipSuccess) {
    sbmm_batch_destroy(b);
    return fail(h, SBMM_E_HIP, "uploading batch tables: %s", hipGetErrorString(e));
  }
  setup_materialized(b, lpm, col_end, colmaps, colscales);
  b->exact_lds = true;
  for (int32_t t = 0; t < T; ++t) b->exact_lds = b->exact_lds && grouped_lds_ok(b->launches[0][t]);
  for (int g = 0; g < kProducts; ++g) {
    for (int i = 0; i < SBMM_BATCH_TUNING_SLOTS; ++i) b->tuning.ms[g][i] = -1.0f;
    if ((st = apply_product(b, g, 0, 1)) != SBMM_OK) {
      sbmm_batch_destroy(b);
      return st;
    }
  }
  *batch = b;
  return SBMM_OK;
}

sbmm_status sbmm_batch_destroy(sbmm_batch b) {
  if (!b) return SBMM_E_ARG;
  // teardown is best effort: the batch is gone whatever these return
  (void)hipSetDevice(b->h->device);
  drop_graph(b);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  if (b->mem) (void)hipFree(b->mem);
  if (b->sk_mem) (void)hipFree(b->sk_mem);
  delete b;
  return SBMM_OK;
}

sbmm_status sbmm_batch_run(sbmm_handle h, sbmm_batch b, sbmm_stream stream) {
  sbmm_status st = check_batch(h, b);
  if (st != SBMM_OK) return st;
  return enqueue_pass(b, (hipStream_t)stream);
}

sbmm_status sbmm_batch_capture(sbmm_handle h, sbmm_batch b) {
  sbmm_status st = check_batch(h, b);
  if (st != SBMM_OK) return st;
  drop_graph(b);
  if (!b->cap_stream) HIP_TRY(h, hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking));
  HIP_TRY(h, hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal));
  st = enqueue_pass(b, b->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(b->cap_stream, &g);
  if (st != SBMM_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(h, SBMM_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  b->graph = g;
  const hipError_t ei = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    b->exec = nullptr;
    drop_graph(b);
    return fail(h, SBMM_E_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  return SBMM_OK;
}

sbmm_status sbmm_batch_replay(sbmm_handle h, sbmm_batch b, sbmm_stream stream) {
  sbmm_status st = check_batch(h, b);
  if (st != SBMM_OK) return st;
  if (!b->exec) return fail(h, SBMM_E_STATE, "no captured graph (call sbmm_batch_capture)");
  HIP_TRY(h, hipGraphLaunch(b->exec, (hipStream_t)stream));
  return SBMM_OK;
}

sbmm_status sbmm_batch_tune(sbmm_handle h, sbmm_batch b, int32_t reps, sbmm_batch_tuning* out,
                            sbmm_stream stream) {
  sbmm_status st = check_batch(h, b);
  if (st != SBMM_OK) return st;
  if (reps < 1) return fail(h, SBMM_E_ARG, "reps must be >= 1");
  hipStream_t s = (hipStream_t)stream;
  drop_graph(b);
  // one full pass so that the sketched product has its plan and MN
  if ((st = enqueue_pass(b, s)) != SBMM_OK) return st;
  hipEvent_t e0, e1;
  HIP_TRY(h, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(h, SBMM_E_HIP, "hipEventCreate");
  }
  st = SBMM_OK;
  for (int g = 0; g < kProducts && st == SBMM_OK; ++g) {
    float best = -1.0f;
    int best_cfg = 0, best_lpt = 1;
    for (int cfg = 0; cfg < product_cfgs(b, g) && st == SBMM_OK; ++cfg)
      for (int lpt = 0; lpt < 2 && st == SBMM_OK && cfg_ok(b, g, cfg); ++lpt) {
        if (hipStreamSynchronize(s) != hipSuccess) { st = fail(h, SBMM_E_HIP, "sync"); break; }
        if ((st = apply_product(b, g, cfg, lpt)) != SBMM_OK) break;
        hipError_t e = enqueue_product(b, g, s);   // warm-up
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = enqueue_product(b, g, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) { st = fail(h, SBMM_E_HIP, "timing: %s", hipGetErrorString(e)); break; }
        ms /= (float)reps;
        b->tuning.ms[g][2 * cfg + lpt] = ms;
        if (best < 0.0f || ms < best) { best = ms; best_cfg = cfg; best_lpt = lpt; }
      }
    if (st == SBMM_OK) st = apply_product(b, g, best_cfg, best_lpt);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != SBMM_OK) return st;
  if (out) *out = b->tuning;
  return SBMM_OK;
}

sbmm_status sbmm_batch_set_tuning(sbmm_handle h, sbmm_batch b, const sbmm_batch_tuning* t) {
  sbmm_status st = check_batch(h, b);
  if (st != SBMM_OK) return st;
  if (!t) return fail(h, SBMM_E_ARG, "tuning is NULL");
  for (int g = 0; g < kProducts; ++g)
    if (!cfg_ok(b, g, t->cfg[g]) || (t->lpt[g] != 0 && t->lpt[g] != 1))
      return fail(h, SBMM_E_ARG, "tuning: configuration out of range");
  HIP_TRY(h, hipDeviceSynchronize());
  drop_graph(b);
  for (int g = 0; g < kProducts; ++g)
    if ((st = apply_product(b, g, t->cfg[g], t->lpt[g])) != SBMM_OK) return st;
  for (int g = 0; g < kProducts; ++g)
    for (int i = 0; i < SBMM_BATCH_TUNING_SLOTS; ++i) b->tuning.ms[g][i] = t->ms[g][i];
  return SBMM_OK;
}

}  // extern "C"
