// C ABI of libsbmm: validation, workspace, stream ordering and status codes
// around the kernels of the sampled block matrix product.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "api_internal.h"

namespace {

// Bump allocator over the handle's workspace. A dry run (base == nullptr)
// only measures; it hands out distinct non-null placeholders (never
// dereferenced: no launch or copy happens in a dry run) so that code which
// decides on whether an optional buffer exists (block norms, pilot
// estimates) sizes itself exactly as the real run does.
struct Arena {
  char* base;
  size_t off = 0;
  explicit Arena(char* b) : base(b) {}
  template <typename T> T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : reinterpret_cast<T*>((uintptr_t)256 + off);
    off += sizeof(T) * (count ? count : 1);
    return p;
  }
};

sbmm_status ensure_ws(sbmm_handle h, size_t bytes) {
  if (bytes <= h->ws_bytes) return SBMM_OK;
  HIP_TRY(h, hipSetDevice(h->device));
  HIP_TRY(h, hipDeviceSynchronize());
  if (h->ws) {
    HIP_TRY(h, hipFree(h->ws));
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = std::max(bytes, (size_t)1 << 20);
  hipError_t e = hipMalloc(&h->ws, want);
  if (e != hipSuccess) {
    h->ws = nullptr;
    (void)hipGetLastError();   // the failed allocation must not surface at the next launch check
    return fail(h, SBMM_E_NOMEM, "workspace of %zu bytes: %s", want, hipGetErrorString(e));
  }
  h->ws_bytes = want;
  return SBMM_OK;
}

bool dtype_in_ok(const sbmm_dtype& t) {
  const int v = enum_raw(t);
  return v == SBMM_F64 || v == SBMM_F32 || v == SBMM_BF16;
}

// Host-side validation of a problem; fills the derived sizes.
sbmm_status validate(sbmm_handle h, const sbmm_problem* P, sbmm_sizes* sz, bool blkprod_internal = false) {
  if (!P) return fail(h, SBMM_E_ARG, "problem is NULL");
  if (P->n < 1 || P->m < 0 || P->p < 0)
    return fail(h, SBMM_E_ARG, "shape m=%lld n=%lld p=%lld (need n >= 1, m, p >= 0)",
                (long long)P->m, (long long)P->n, (long long)P->p);
  if (P->n > INT32_MAX) return fail(h, SBMM_E_ARG, "n exceeds 2^31 - 1");
  if (!dtype_in_ok(P->in_dtype)) return fail(h, SBMM_E_ARG, "input dtype %d not supported", enum_raw(P->in_dtype));
  const uintptr_t es = (uintptr_t)dtype_size(P->in_dtype);
  if ((P->m > 0 && (uintptr_t)P->M % es) || (P->p > 0 && (uintptr_t)P->N % es))
    return fail(h, SBMM_E_ARG, "M or N is not aligned to its %d-byte elements", (int)es);
  if (P->m > 0 && (!P->M || P->ldm < P->n))
    return fail(h, SBMM_E_ARG, "M is NULL or ldm < n");
  if (P->p > 0 && (!P->N || P->ldn < P->p))
    return fail(h, SBMM_E_ARG, "N is NULL or ldn < p");
  if (P->K < 1 || !P->block_off) return fail(h, SBMM_E_ARG, "need K >= 1 and block offsets");
  if (P->block_off[0] != 0 || P->block_off[P->K] != P->n)
    return fail(h, SBMM_E_ARG, "block offsets must start at 0 and end at n");
  int64_t maxw = 0;
  for (int32_t k = 0; k < P->K; ++k) {
    const int64_t w = P->block_off[k + 1] - P->block_off[k];
    if (w < 1) return fail(h, SBMM_E_ARG, "block %d has size %lld (need >= 1)", k, (long long)w);
    maxw = std::max(maxw, w);
  }
  if (P->c < 1 || P->c > INT32_MAX) return fail(h, SBMM_E_ARG, "c = %lld out of range", (long long)P->c);
  if (enum_raw(P->mode) != SBMM_MODE_BLOCK && enum_raw(P->mode) != SBMM_MODE_STRATIFIED)
    return fail(h, SBMM_E_ARG, "unknown mode %d", enum_raw(P->mode));
  if (enum_raw(P->prob) < SBMM_P_UNIFORM || enum_raw(P->prob) > SBMM_P_USER)
    return fail(h, SBMM_E_ARG, "unknown probability rule %d", enum_raw(P->prob));
  if (P->prob == SBMM_P_USER && !P->user_w) return fail(h, SBMM_E_ARG, "rule USER needs user_w");
  if (P->mode == SBMM_MODE_BLOCK) {
    if (P->prob == SBMM_P_EXACT && !P->blkprod_sq && !blkprod_internal)
      return fail(h, SBMM_E_ARG, "rule EXACT needs blkprod_sq (from sbmm_exact)");
  } else {
    if (enum_raw(P->alloc) < SBMM_ALLOC_UNIFORM || enum_raw(P->alloc) > SBMM_ALLOC_TWO_STEP)
      return fail(h, SBMM_E_ARG, "unknown allocation rule %d", enum_raw(P->alloc));
    if (P->alloc == SBMM_ALLOC_OPT && !P->blkprod_sq && !blkprod_internal)
      return fail(h, SBMM_E_ARG, "allocation OPT needs blkprod_sq (from sbmm_exact)");
    if (P->alloc == SBMM_ALLOC_TWO_STEP && !P->pilot_sq && !blkprod_internal)
      return fail(h, SBMM_E_ARG, "allocation TWO_STEP needs pilot_sq (from sbmm_pilot)");
    if (P->alloc == SBMM_ALLOC_USER) {
      if (!P->user_ck) return fail(h, SBMM_E_ARG, "allocation USER needs user_ck");
      int64_t s = 0;
      for (int32_t k = 0; k < P->K; ++k) {
        if (P->user_ck[k] < 0) return fail(h, SBMM_E_ARG, "user_ck[%d] < 0", k);
        s += P->user_ck[k];
      }
      if (s != P->c) return fail(h, SBMM_E_ARG, "user_ck sums to %lld, not c = %lld", (long long)s, (long long)P->c);
    }
  }
  if (sz) {
    const bool blockm = P->mode == SBMM_MODE_BLOCK;
    sz->atoms = blockm ? P->K : P->n;
    sz->strata = blockm ? 1 : P->K;
    sz->max_width = blockm ? maxw : 1;
    sz->L_max = P->c * sz->max_width;
    sz->L_pad_max = round_up(sz->L_max, SBMM_SKETCH_PAD);
  }
  return SBMM_OK;
}

// The pilot's parameters (Alg. 3 step 1): stratified mode, [c0/K] >= 1
// draws per block, uniform or (3.8) probabilities.
sbmm_status validate_pilot(sbmm_handle h, const sbmm_problem* P) {
  if (P->mode != SBMM_MODE_STRATIFIED) return fail(h, SBMM_E_ARG, "the pilot needs stratified mode");
  if (P->c0 < P->K || P->c0 > INT32_MAX)
    return fail(h, SBMM_E_ARG, "c0 = %lld must be at least K = %d (and below 2^31)", (long long)P->c0, P->K);
  if (enum_raw(P->pilot_prob) != SBMM_P_UNIFORM && enum_raw(P->pilot_prob) != SBMM_P_NORM)
    return fail(h, SBMM_E_ARG, "pilot probabilities must be UNIFORM or NORM");
  return SBMM_OK;
}

// the effective probability rule (EXACT on unit atoms is NORM)
int eff_prob(const sbmm_problem* P) {
  if (P->mode == SBMM_MODE_STRATIFIED && P->prob == SBMM_P_EXACT) return SBMM_P_NORM;
  return P->prob;
}

bool needs_blkprod(const sbmm_problem* P) {
  return (P->mode == SBMM_MODE_BLOCK && P->prob == SBMM_P_EXACT) ||
         (P->mode == SBMM_MODE_STRATIFIED && P->alloc == SBMM_ALLOC_OPT);
}

// --- internal steps (work on an arena that already has room) --------------

// The device copy of the problem's block offsets. The handle keeps the last
// partition it uploaded and enqueues a copy only when the partition differs
// (the copy is ordered on `s` after the work already enqueued there). A dry
// run gets a placeholder and no copy.
sbmm_status upload_offsets(sbmm_handle h, const sbmm_problem* P, Arena& ar, int64_t** out, hipStream_t s) {
  const size_t cnt = (size_t)P->K + 1;
  if (!ar.base) {
    *out = reinterpret_cast<int64_t*>((uintptr_t)256);
    return SBMM_OK;
  }
  if (h->off_dev && h->off_host.size() == cnt &&
      std::memcmp(h->off_host.data(), P->block_off, sizeof(int64_t) * cnt) == 0) {
    *out = h->off_dev;
    return SBMM_OK;
  }
  if (cnt > h->off_cap) {
    HIP_TRY(h, hipDeviceSynchronize());   // earlier work may still read the old copy
    if (h->off_dev) HIP_TRY(h, hipFree(h->off_dev));
    h->off_dev = nullptr;
    h->off_cap = 0;
    h->off_host.clear();
    const size_t cap = std::max(cnt, (size_t)1024);
    hipError_t e = hipMalloc(&h->off_dev, sizeof(int64_t) * cap);
    if (e != hipSuccess) {
      h->off_dev = nullptr;
      (void)hipGetLastError();
      return fail(h, SBMM_E_NOMEM, "block offsets: %s", hipGetErrorString(e));
    }
    h->off_cap = cap;
  }
  h->off_host.clear();   // stale until the copy is enqueued
  HIP_TRY(h, hipMemcpyAsync(h->off_dev, P->block_off, sizeof(int64_t) * cnt, hipMemcpyHostToDevice, s));
  h->off_host.assign(P->block_off, P->block_off + cnt);
  *out = h->off_dev;
  return SBMM_OK;
}

int64_t max_block_width(const sbmm_problem* P) {
  int64_t w = 0;
  for (int32_t k = 0; k < P->K; ++k) w = std::max(w, P->block_off[k + 1] - P->block_off[k]);
  return w;
}

sbmm_status do_norms(sbmm_handle h, const sbmm_problem* P, const int64_t* off_dev, double* col_sq,
                     double* row_sq, double* blk, Arena& ar, hipStream_t s) {
  int R = 1;
  const size_t pe = norms_partial_elems(P->in_dtype, P->m, P->n, &R);
  double* partial = ar.take<double>(pe);
  const int32_t chunks = norms_stats_chunks(P->n, P->K, max_block_width(P));
  double* stats_part = chunks > 1 ? ar.take<double>(3 * (size_t)P->K * chunks) : nullptr;
  if (!ar.base) return SBMM_OK;
  NormLaunch L{};
  L.dt = P->in_dtype; L.M = P->M; L.ldm = P->ldm; L.N = P->N; L.ldn = P->ldn;
  L.m = P->m; L.n = P->n; L.p = P->p; L.K = P->K; L.off_dev = off_dev;
  L.partial = partial; L.rsplit = R; L.col_sq = col_sq; L.row_sq = row_sq; L.blk = blk;
  L.status = h->status; L.stats_chunks = chunks; L.stats_part = stats_part;
  HIP_TRY(h, launch_norms(L, s));
  return SBMM_OK;
}

sbmm_dtype product_dtype(sbmm_dtype in) { return in == SBMM_F64 ? SBMM_F64 : SBMM_F32; }

// launch_gemm, or its split-K form when the caller sized a workspace for it.
hipError_t run_product(const GemmLaunch& G, hipStream_t s) {
  if (G.skinny_ws) {
    const int64_t tiles = gemm_tiles(G.dt, G.m, G.p, G.blk_part != nullptr);
    return launch_gemm_skinny(G, tiles, tiles * 4, s);
  }
  return launch_gemm(G, s);
}

// Exact product with optional MN store, block norms and error vs Y.
// Block norms of float32 and bf16 problems with blocks up to 128 wide come
// from the Gram-matrix kernel (cheap, separate launch); otherwise the float32
// product kernel accumulates them block by block (bf16 inputs promoted
// exactly to float32 copies in the workspace first).
sbmm_status do_exact(sbmm_handle h, const sbmm_problem* P, const int64_t* off_dev, void* MN, int64_t ldmn,
                     const void* Y, int64_t ldy, double* blkprod_sq, double* out2, Arena& ar, hipStream_t s) {
  const int64_t wmax = max_block_width(P);
  const bool gram = blkprod_sq != nullptr && (P->in_dtype == SBMM_F32 || P->in_dtype == SBMM_BF16) &&
                    wmax <= block_gram_max_width() && block_gram_strides_ok(P->ldm, P->ldn);
  if (gram) {
    void* gws = ar.take<char>(block_gram_ws_bytes(P->K, wmax));
    if (ar.base) {
      if (P->m > 0 && P->p > 0) {
        HIP_TRY(h, launch_block_gram(P->in_dtype, P->M, P->ldm, P->N, P->ldn, P->m, P->p, off_dev, P->K, wmax,
                                     blkprod_sq, gws, s));
      } else {
        HIP_TRY(h, launch_fill_f64(blkprod_sq, P->K, 0.0, s));
      }
    }
    blkprod_sq = nullptr;   // the product kernel below needs no block bookkeeping
  }
  if (P->in_dtype == SBMM_BF16 && blkprod_sq) {
    // wide blocks of a bf16 problem: the float32 product with per-block sums
    // over exact float32 copies of M and N
    sbmm_problem Q = *P;
    float* M32 = ar.take<float>((size_t)P->m * P->n);
    float* N32 = ar.take<float>((size_t)P->n * P->p);
    if (ar.base) {
      HIP_TRY(h, launch_bf16_to_f32(reinterpret_cast<const uint16_t*>(P->M), P->m, P->n, P->ldm, M32, P->n, s));
      HIP_TRY(h, launch_bf16_to_f32(reinterpret_cast<const uint16_t*>(P->N), P->n, P->p, P->ldn, N32, P->p, s));
    }
    Q.in_dtype = SBMM_F32;
    Q.M = M32; Q.ldm = P->n; Q.N = N32; Q.ldn = P->p;
    return do_exact(h, &Q, off_dev, MN, ldmn, Y, ldy, blkprod_sq, out2, ar, s);
  }
  const bool bn = blkprod_sq != nullptr;
  GemmLaunch G{};
  G.dt = P->in_dtype; G.A = P->M; G.lda = P->ldm; G.B = P->N; G.ldb = P->ldn;
  G.m = P->m; G.p = P->p; G.K_host = P->n; G.K_dev = nullptr;
  // bf16 products never carry block sums here (handled above)
  const int64_t tiles = P->in_dtype == SBMM_BF16 ? hgemm_tiles(G) : gemm_tiles(P->in_dtype, P->m, P->p, bn);
  double* tile_part = ar.take<double>(2 * std::max<int64_t>(tiles, 1));
  double* blk_part = bn ? ar.take<double>((size_t)P->K * std::max<int64_t>(tiles, 1) * 4) : nullptr;
  float* stage = ar.take<float>(gemm_stage_bytes(P->in_dtype, P->m, P->p) / sizeof(float));
  const size_t skb = gemm_skinny_ws_bytes(P->in_dtype, P->m, P->p, P->n, bn ? P->K : 0);
  void* skinny = skb ? ar.take<char>(skb) : nullptr;
  if (!ar.base) return SBMM_OK;
  if (tiles == 0) {
    HIP_TRY(h, launch_fill_f64(out2, 2, 0.0, s));
    if (bn) HIP_TRY(h, launch_fill_f64(blkprod_sq, P->K, 0.0, s));
    return SBMM_OK;
  }
  G.Cout = MN; G.ldc = ldmn; G.Y = Y; G.ldy = ldy; G.tile_part = tile_part;
  G.K_blocks = P->K; G.off_dev = off_dev; G.blk_part = blk_part; G.stage = stage;
  G.skinny_ws = skinny; G.skinny_K_max = P->n;
  HIP_TRY(h, run_product(G, s));
  HIP_TRY(h, launch_reduce_cols(tile_part, 2, tiles, out2, s));
  if (bn) HIP_TRY(h, launch_reduce_cols(blk_part, P->K, tiles * 4, blkprod_sq, s));
  return SBMM_OK;
}

sbmm_status do_plan(sbmm_handle h, const sbmm_problem* P, const sbmm_sizes& sz, const int64_t* off_dev,
                    const double* col_sq, const double* row_sq, const double* blk, const sbmm_plan_out* out,
                    Arena& ar, hipStream_t s, int64_t pilot_r = 0, int64_t** draw_off_out = nullptr) {
  PlanLaunch L{};
  L.W = ar.take<uint64_t>(sz.atoms);
  L.cdf = ar.take<uint64_t>(sz.atoms);
  L.T = ar.take<uint64_t>(sz.strata);
  L.draw_off = ar.take<int64_t>(sz.strata + 1);
  L.width = ar.take<int64_t>(P->c);
  L.G = ar.take<uint64_t>(sz.strata);
  L.quota = ar.take<int64_t>(sz.strata);
  L.rem = ar.take<uint64_t>(sz.strata);
  L.left = ar.take<int64_t>(1);
  int64_t* user_ck_dev = nullptr;
  const bool uck = P->mode == SBMM_MODE_STRATIFIED && P->alloc == SBMM_ALLOC_USER && pilot_r == 0;
  if (uck) user_ck_dev = ar.take<int64_t>(P->K);
  const int64_t max_atoms = P->mode == SBMM_MODE_BLOCK ? P->K : max_block_width(P);
  L.dchunks = plan_design_chunks(max_atoms, sz.atoms, sz.strata);
  if (L.dchunks > 1) {
    L.dpart_max = ar.take<double>((size_t)sz.strata * L.dchunks);
    L.dpart_sum = ar.take<uint64_t>((size_t)sz.strata * L.dchunks);
  }
  if (plan_wide_offsets(P->c)) L.wpart = ar.take<uint64_t>(ceil_div(P->c, 256));
  if (draw_off_out) *draw_off_out = L.draw_off;
  if (!ar.base) return SBMM_OK;
  if (uck) HIP_TRY(h, hipMemcpyAsync(user_ck_dev, P->user_ck, sizeof(int64_t) * P->K, hipMemcpyHostToDevice, s));
  // alloc is read only in stratified mode (a block problem may leave it unset)
  L.mode = P->mode; L.prob = eff_prob(P);
  L.alloc = P->mode == SBMM_MODE_STRATIFIED ? P->alloc : SBMM_ALLOC_UNIFORM;
  L.n = P->n; L.K = P->K; L.c = P->c; L.A = sz.atoms; L.S = sz.strata;
  L.off_dev = off_dev; L.col_sq = col_sq; L.row_sq = row_sq; L.blk = blk;
  L.user_w = P->user_w; L.user_ck_dev = user_ck_dev; L.blkprod_sq = P->blkprod_sq;
  L.pilot_sq = P->pilot_sq; L.pilot_r = pilot_r;
  L.seed = P->seed; L.trial = P->trial;
  L.idx = out->idx; L.scale = out->scale; L.col_off = out->col_off; L.ck = out->ck;
  L.p_hat = out->p_hat; L.colmap = out->colmap; L.colscale = out->colscale;
  L.L_pad_max = sz.L_pad_max; L.status = h->status;
  HIP_TRY(h, launch_plan(L, s));
  return SBMM_OK;
}

bool plan_out_ok(const sbmm_plan_out* o) {
  return o && o->idx && o->scale && o->col_off && o->ck && o->colmap && o->colscale;
}

bool sketch_dtype_ok(const sbmm_dtype& in, const sbmm_dtype& out) {
  const int i = enum_raw(in), o = enum_raw(out);
  if (i == SBMM_F64) return o == SBMM_F64;
  return (i == SBMM_F32 || i == SBMM_BF16) && (o == SBMM_F32 || o == SBMM_BF16);
}

// Alg. 3 step 1: the pilot plan ([c0/K] draws per block, tag 2), its sketch
// C0 (m x round_up(c0, 32)) and D0 in the product dtype, and per block the
// squared Frobenius norm of C^{0k} D_{0k}, by the block-norm form of the
// product kernel with the strata's column ranges (draw offsets: pilot draws
// are single columns) as the blocks. `pp` (may be NULL) receives the draws.
sbmm_status do_pilot(sbmm_handle h, const sbmm_problem* P, const int64_t* off_dev, const double* col_sq,
                     const double* row_sq, const double* blk, const sbmm_plan_out* pp, double* pilot_sq,
                     Arena& ar, hipStream_t s) {
  sbmm_problem Q = *P;
  Q.prob = P->pilot_prob;
  Q.c = P->c0;
  Q.alloc = SBMM_ALLOC_UNIFORM;   // not used: the pilot counts are fixed
  sbmm_sizes sz;
  sz.atoms = P->n;
  sz.strata = P->K;
  sz.max_width = 1;
  sz.L_max = P->c0;
  sz.L_pad_max = round_up(P->c0, SBMM_SKETCH_PAD);
  const int64_t Lp = sz.L_pad_max;
  sbmm_plan_out own{};
  if (!pp) {
    own.idx = ar.take<int32_t>(Q.c);
    own.scale = ar.take<double>(Q.c);
    own.col_off = ar.take<int64_t>(Q.c + 1);
    own.ck = ar.take<int64_t>(P->K);
    own.colmap = ar.take<int32_t>(Lp);
    own.colscale = ar.take<double>(Lp);
    pp = &own;
  }
  const sbmm_dtype pd = product_dtype(P->in_dtype);
  const size_t es = dtype_size(pd);
  void* C0 = ar.take<char>(es * (size_t)std::max<int64_t>(P->m, 1) * Lp);
  void* D0 = ar.take<char>(es * (size_t)Lp * std::max<int64_t>(P->p, 1));
  const int64_t tiles = gemm_tiles(pd, P->m, P->p, true);
  double* tile_part = ar.take<double>(2 * std::max<int64_t>(tiles, 1));
  double* blk_part = ar.take<double>((size_t)P->K * std::max<int64_t>(tiles, 1) * 4);
  const size_t skb = gemm_skinny_ws_bytes(pd, P->m, P->p, Lp, P->K);
  void* skinny = skb ? ar.take<char>(skb) : nullptr;
  int64_t* draw_off = nullptr;
  sbmm_status st = do_plan(h, &Q, sz, off_dev, col_sq, row_sq, blk, pp, ar, s, P->c0 / P->K, &draw_off);
  if (st || !ar.base) return st;
  if (tiles == 0) {
    HIP_TRY(h, launch_fill_f64(pilot_sq, P->K, 0.0, s));
    return SBMM_OK;
  }
  GatherLaunch g{};
  g.in_dt = P->in_dtype; g.out_dt = pd;
  g.M = P->M; g.ldm = P->ldm; g.N = P->N; g.ldn = P->ldn; g.m = P->m; g.p = P->p;
  g.L_dev = pp->col_off + Q.c; g.L_pad_max = Lp;
  g.colmap = pp->colmap; g.colscale = pp->colscale;
  g.C = C0; g.ldc = Lp; g.D = D0; g.ldd = P->p;
  HIP_TRY(h, launch_gather(g, s));
  GemmLaunch G{};
  G.dt = pd; G.A = C0; G.lda = Lp; G.B = D0; G.ldb = P->p; G.m = P->m; G.p = P->p;
  G.K_host = 0; G.K_dev = pp->col_off + Q.c; G.Cout = nullptr; G.ldc = P->p;
  G.Y = nullptr; G.ldy = P->p; G.tile_part = tile_part;
  G.K_blocks = P->K; G.off_dev = draw_off; G.blk_part = blk_part; G.stage = nullptr;
  G.skinny_ws = skinny; G.skinny_K_max = Lp;
  HIP_TRY(h, run_product(G, s));
  HIP_TRY(h, launch_reduce_cols(blk_part, P->K, tiles * 4, pilot_sq, s));
  return SBMM_OK;
}

}  // namespace

// ============================================================================
// Public entry points
// ============================================================================

// Fixed scratch of sbmm_plan_noalloc, one copy per GPU, held until the
// process ends. Host code never uses this name as an address: each device's
// copy is found once with hipGetSymbolAddress (with that device current) and
// that pointer is what the kernels receive.
static __device__ __align__(256) char scratch[SBMM_NOALLOC_SCRATCH_BYTES];

namespace {

std::mutex g_scratch_mu;
std::vector<char*> g_scratch_dev;   // indexed by device; nullptr until bound

sbmm_status bind_scratch(sbmm_handle h) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev.size() <= (size_t)h->device) g_scratch_dev.resize((size_t)h->device + 1, nullptr);
  if (!g_scratch_dev[h->device]) {
    char* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(h, SBMM_E_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_dev[h->device] = ptr;
  }
  h->scratch = g_scratch_dev[h->device];
  return SBMM_OK;
}

}  // namespace

extern "C" {

const char* sbmm_status_string(sbmm_status s) {
  switch (enum_raw(s)) {
    case SBMM_OK: return "ok";
    case SBMM_E_ARG: return "invalid argument";
    case SBMM_E_BUDGET: return "sample budget too small";
    case SBMM_E_NONFINITE: return "non-finite input";
    case SBMM_E_UNSUPPORTED: return "unsupported";
    case SBMM_E_NOMEM: return "out of device memory";
    case SBMM_E_HIP: return "HIP error";
    case SBMM_E_STATE: return "invalid handle state";
  }
  return "unknown status";
}

sbmm_status sbmm_create(sbmm_handle* out, int device) {
  if (!out) return SBMM_E_ARG;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) return SBMM_E_ARG;
  sbmm_handle h = new (std::nothrow) sbmm_handle_s();
  if (!h) return SBMM_E_NOMEM;
  h->device = device;
  if (hipSetDevice(device) != hipSuccess) { delete h; return SBMM_E_HIP; }
  if (hipMalloc(&h->status, sizeof(int32_t)) != hipSuccess) { delete h; return SBMM_E_NOMEM; }
  const int32_t zero = 0;
  if (hipMemcpy(h->status, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(h->status);
    delete h;
    return SBMM_E_HIP;
  }
  // room for the partition of up to 1023 blocks
  if (hipMalloc(&h->off_dev, sizeof(int64_t) * 1024) != hipSuccess) {
    (void)hipFree(h->status);
    delete h;
    return SBMM_E_NOMEM;
  }
  h->off_cap = 1024;
  if (bind_scratch(h) != SBMM_OK) {
    (void)hipFree(h->off_dev);
    (void)hipFree(h->status);
    delete h;
    return SBMM_E_HIP;
  }
  *out = h;
  return SBMM_OK;
}

sbmm_status sbmm_destroy(sbmm_handle h) {
  if (!h) return SBMM_E_STATE;
  // teardown is best effort: the handle is gone whatever these return
  (void)hipSetDevice(h->device);
  if (h->ws) (void)hipFree(h->ws);
  if (h->off_dev) (void)hipFree(h->off_dev);
  if (h->status) (void)hipFree(h->status);
  h->status = nullptr;
  delete h;
  return SBMM_OK;
}

const char* sbmm_last_error(sbmm_handle h) { return h ? h->err : "null handle"; }

sbmm_status sbmm_reserve(sbmm_handle h, size_t bytes) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  return ensure_ws(h, bytes);
}

sbmm_status sbmm_sync(sbmm_handle h, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  return read_status(h, (hipStream_t)stream);
}

sbmm_status sbmm_query_sizes(const sbmm_problem* prob, sbmm_sizes* out) {
  if (!out) return SBMM_E_ARG;
  return validate(nullptr, prob, out, true);   // sizes do not depend on blkprod_sq
}

sbmm_status sbmm_norms(sbmm_handle h, const sbmm_problem* P, double* col_sq, double* row_sq, double* blk,
                       sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  sbmm_sizes sz;
  if ((st = validate(h, P, &sz, true))) return st;
  if (!col_sq || !row_sq || !blk) return fail(h, SBMM_E_ARG, "col_sq, row_sq and blk are required");
  hipStream_t s = (hipStream_t)stream;
  Arena dry(nullptr);
  int64_t* off = nullptr;
  upload_offsets(h, P, dry, &off, s);
  do_norms(h, P, off, col_sq, row_sq, blk, dry, s);
  if ((st = ensure_ws(h, dry.off))) return st;
  Arena ar(h->ws);
  if ((st = upload_offsets(h, P, ar, &off, s))) return st;
  return do_norms(h, P, off, col_sq, row_sq, blk, ar, s);
}

sbmm_status sbmm_exact(sbmm_handle h, const sbmm_problem* P, void* MN, int64_t ldmn, double* blkprod_sq,
                       double* mn_sq, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  sbmm_sizes sz;
  if ((st = validate(h, P, &sz, true))) return st;
  if (!mn_sq) return fail(h, SBMM_E_ARG, "mn_sq is required");
  if (MN && ldmn < P->p) return fail(h, SBMM_E_ARG, "ldmn < p");
  hipStream_t s = (hipStream_t)stream;
  Arena dry(nullptr);
  int64_t* off = nullptr;
  upload_offsets(h, P, dry, &off, s);
  double* out2 = dry.take<double>(2);
  if ((st = do_exact(h, P, off, MN, ldmn, nullptr, 0, blkprod_sq, out2, dry, s))) return st;
  if ((st = ensure_ws(h, dry.off))) return st;
  Arena ar(h->ws);
  if ((st = upload_offsets(h, P, ar, &off, s))) return st;
  out2 = ar.take<double>(2);
  if ((st = do_exact(h, P, off, MN, ldmn, nullptr, 0, blkprod_sq, out2, ar, s))) return st;
  HIP_TRY(h, hipMemcpyAsync(mn_sq, out2 + 1, sizeof(double), hipMemcpyDeviceToDevice, s));
  return SBMM_OK;
}

// Argument checks shared by sbmm_plan and sbmm_plan_noalloc.
static sbmm_status plan_args(sbmm_handle h, const sbmm_problem* P, const double* col_sq, const double* row_sq,
                      const double* blk, const sbmm_plan_out* out, sbmm_sizes* sz) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  if ((st = validate(h, P, sz))) return st;
  if (!plan_out_ok(out)) return fail(h, SBMM_E_ARG, "plan output buffers missing");
  const int pr = eff_prob(P);
  const bool strat = P->mode == SBMM_MODE_STRATIFIED;
  const bool need_blk = (!strat && pr == SBMM_P_NORM) ||
                        (strat && (P->alloc == SBMM_ALLOC_NORM || P->alloc == SBMM_ALLOC_OPT ||
                                   P->alloc == SBMM_ALLOC_TWO_STEP));
  if (strat && P->alloc == SBMM_ALLOC_TWO_STEP && (st = validate_pilot(h, P))) return st;
  const bool need_colrow = strat && pr == SBMM_P_NORM;
  if ((need_blk && !blk) || (need_colrow && (!col_sq || !row_sq)))
    return fail(h, SBMM_E_ARG, "the rule needs the norm-pass outputs");
  return SBMM_OK;
}

sbmm_status sbmm_plan(sbmm_handle h, const sbmm_problem* P, const double* col_sq, const double* row_sq,
                      const double* blk, const sbmm_plan_out* out, int64_t* L_host, sbmm_stream stream) {
  sbmm_sizes sz;
  sbmm_status st = plan_args(h, P, col_sq, row_sq, blk, out, &sz);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  Arena dry(nullptr);
  int64_t* off = nullptr;
  upload_offsets(h, P, dry, &off, s);
  do_plan(h, P, sz, off, col_sq, row_sq, blk, out, dry, s);
  if ((st = ensure_ws(h, dry.off))) return st;
  Arena ar(h->ws);
  if ((st = upload_offsets(h, P, ar, &off, s))) return st;
  if ((st = do_plan(h, P, sz, off, col_sq, row_sq, blk, out, ar, s))) return st;
  if (L_host) {
    HIP_TRY(h, hipMemcpyAsync(L_host, out->col_off + P->c, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    return read_status(h, s);
  }
  return SBMM_OK;
}

// The same plan with every scratch buffer, the device copy of the partition
// included, in the GPU's fixed scratch array: no workspace growth, no
// allocation. The dry pass measures the layout the real pass takes.
sbmm_status sbmm_plan_noalloc(sbmm_handle h, const sbmm_problem* P, const double* col_sq, const double* row_sq,
                              const double* blk, const sbmm_plan_out* out, int64_t* L_host, sbmm_stream stream) {
  sbmm_sizes sz;
  sbmm_status st = plan_args(h, P, col_sq, row_sq, blk, out, &sz);
  if (st) return st;
  if (!h->scratch) return fail(h, SBMM_E_STATE, "the fixed scratch array of device %d is not bound", h->device);
  hipStream_t s = (hipStream_t)stream;
  Arena dry(nullptr);
  int64_t* off = dry.take<int64_t>((size_t)P->K + 1);
  do_plan(h, P, sz, off, col_sq, row_sq, blk, out, dry, s);
  if (dry.off > (size_t)SBMM_NOALLOC_SCRATCH_BYTES)
    return fail(h, SBMM_E_ARG, "the plan needs %zu bytes of scratch, above the fixed %zu of sbmm_plan_noalloc",
                dry.off, (size_t)SBMM_NOALLOC_SCRATCH_BYTES);
  Arena ar(h->scratch);
  off = ar.take<int64_t>((size_t)P->K + 1);
  HIP_TRY(h, hipMemcpyAsync(off, P->block_off, sizeof(int64_t) * ((size_t)P->K + 1), hipMemcpyHostToDevice, s));
  if ((st = do_plan(h, P, sz, off, col_sq, row_sq, blk, out, ar, s))) return st;
  if (L_host) {
    HIP_TRY(h, hipMemcpyAsync(L_host, out->col_off + P->c, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    return read_status(h, s);
  }
  return SBMM_OK;
}

sbmm_status sbmm_pilot(sbmm_handle h, const sbmm_problem* P, const double* col_sq, const double* row_sq,
                       const double* blk, const sbmm_plan_out* pilot_plan, double* pilot_sq, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  if ((st = validate(h, P, nullptr, true))) return st;
  if ((st = validate_pilot(h, P))) return st;
  if (!pilot_sq) return fail(h, SBMM_E_ARG, "pilot_sq is required");
  if (pilot_plan && !plan_out_ok(pilot_plan)) return fail(h, SBMM_E_ARG, "pilot plan buffers missing");
  if (P->pilot_prob == SBMM_P_NORM && (!col_sq || !row_sq))
    return fail(h, SBMM_E_ARG, "NORM pilot probabilities need col_sq and row_sq");
  hipStream_t s = (hipStream_t)stream;
  Arena dry(nullptr);
  int64_t* off = nullptr;
  upload_offsets(h, P, dry, &off, s);
  do_pilot(h, P, off, col_sq, row_sq, blk, pilot_plan, pilot_sq, dry, s);
  if ((st = ensure_ws(h, dry.off))) return st;
  Arena ar(h->ws);
  if ((st = upload_offsets(h, P, ar, &off, s))) return st;
  return do_pilot(h, P, off, col_sq, row_sq, blk, pilot_plan, pilot_sq, ar, s);
}

sbmm_status sbmm_sketch(sbmm_handle h, const sbmm_problem* P, const sbmm_plan_out* plan, sbmm_dtype out_dtype,
                        void* C, int64_t ldc, void* D, int64_t ldd, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  sbmm_sizes sz;
  if ((st = validate(h, P, &sz, true))) return st;
  if (!plan || !plan->col_off || !plan->colmap || !plan->colscale) return fail(h, SBMM_E_ARG, "plan buffers missing");
  if (!sketch_dtype_ok(P->in_dtype, out_dtype)) return fail(h, SBMM_E_ARG, "sketch dtype not allowed for the input dtype");
  if (C && ldc < sz.L_pad_max) return fail(h, SBMM_E_ARG, "ldc < L_pad_max (%lld)", (long long)sz.L_pad_max);
  if (D && ldd < P->p) return fail(h, SBMM_E_ARG, "ldd < p");
  GatherLaunch g{};
  g.in_dt = P->in_dtype; g.out_dt = out_dtype;
  g.M = P->M; g.ldm = P->ldm; g.N = P->N; g.ldn = P->ldn; g.m = P->m; g.p = P->p;
  g.L_dev = plan->col_off + P->c; g.L_pad_max = sz.L_pad_max;
  g.colmap = plan->colmap; g.colscale = plan->colscale;
  g.C = C; g.ldc = ldc; g.D = D; g.ldd = ldd;
  HIP_TRY(h, launch_gather(g, (hipStream_t)stream));
  return SBMM_OK;
}

sbmm_status sbmm_sketch_gemm(sbmm_handle h, int64_t m, int64_t p, int64_t L_pad_max, const int64_t* L_dev,
                             sbmm_dtype dtype, const void* C, int64_t ldc, const void* D, int64_t ldd, void* CD,
                             int64_t ldcd, const void* MN, int64_t ldmn, double* err_sq, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  if (m < 0 || p < 0 || L_pad_max < 0 || !L_dev) return fail(h, SBMM_E_ARG, "bad sizes or L_dev");
  if (enum_raw(dtype) != SBMM_F64 && enum_raw(dtype) != SBMM_F32 && enum_raw(dtype) != SBMM_BF16)
    return fail(h, SBMM_E_UNSUPPORTED, "sketched product in dtype %d is not built", enum_raw(dtype));
  if (m > 0 && p > 0 && L_pad_max > 0 && (!C || !D)) return fail(h, SBMM_E_ARG, "C and D are required");
  if (ldc < L_pad_max || ldd < p) return fail(h, SBMM_E_ARG, "ldc < L_pad_max or ldd < p");
  if (CD && ldcd < p) return fail(h, SBMM_E_ARG, "ldcd < p");
  if ((MN != nullptr) != (err_sq != nullptr)) return fail(h, SBMM_E_ARG, "MN and err_sq go together");
  if (MN && ldmn < p) return fail(h, SBMM_E_ARG, "ldmn < p");
  hipStream_t s = (hipStream_t)stream;
  GemmLaunch G{};
  G.dt = dtype; G.A = C; G.lda = ldc; G.B = D; G.ldb = ldd; G.m = m; G.p = p;
  G.K_host = 0; G.K_dev = L_dev; G.K_max = L_pad_max; G.Cout = CD; G.ldc = ldcd; G.Y = MN; G.ldy = ldmn;
  // bf16 reads D as it is where its rows allow (16-byte aligned, 32-bit
  // offsets), otherwise from a transposed copy D^T (p x L_pad)
  const bool bf = dtype == SBMM_BF16;
  const bool bf_t = bf && !hgemm_kn_ok(G);
  const int64_t tiles = bf ? gemm_tiles_tn(m, p) : gemm_tiles(dtype, m, p, false);
  const size_t stage_elems = gemm_stage_bytes(dtype, m, p) / sizeof(float);
  const size_t dt_elems = bf_t ? (size_t)std::max<int64_t>(p, 1) * std::max<int64_t>(L_pad_max, 1) : 0;
  const size_t skb = bf ? 0 : gemm_skinny_ws_bytes(dtype, m, p, L_pad_max, 0);
  Arena dry(nullptr);
  dry.take<double>(2 * std::max<int64_t>(tiles, 1));
  dry.take<float>(stage_elems);
  dry.take<uint16_t>(dt_elems);
  dry.take<char>(skb);
  if ((st = ensure_ws(h, dry.off))) return st;
  Arena ar(h->ws);
  double* tile_part = ar.take<double>(2 * std::max<int64_t>(tiles, 1));
  float* stage = ar.take<float>(stage_elems);
  uint16_t* Dt = ar.take<uint16_t>(dt_elems);
  void* skinny = skb ? ar.take<char>(skb) : nullptr;
  if (tiles == 0) {
    if (err_sq) HIP_TRY(h, launch_fill_f64(err_sq, 1, 0.0, s));
    return SBMM_OK;
  }
  G.tile_part = err_sq ? tile_part : nullptr;
  G.stage = stage;
  if (bf_t) {
    HIP_TRY(h, launch_transpose_bf16(SBMM_BF16, D, L_pad_max, p, ldd, L_dev, Dt, L_pad_max, s));
    G.B = Dt; G.ldb = L_pad_max; G.b_trans = true;
  }
  G.skinny_ws = skinny; G.skinny_K_max = L_pad_max;
  HIP_TRY(h, run_product(G, s));
  if (err_sq) {
    // the squared-error partials (row 0 of tile_part) summed straight into
    // err_sq: one small kernel, no device-to-device copy behind it
    HIP_TRY(h, launch_reduce_cols(tile_part, 1, tiles, err_sq, s));
  }
  return SBMM_OK;
}

sbmm_status sbmm_sketch_mx(sbmm_handle h, const sbmm_problem* P, const sbmm_plan_out* plan, void* C, int64_t ldc,
                           void* Cs, int64_t ldcs, void* Dt, int64_t lddt, void* Ds, int64_t ldds,
                           sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  sbmm_sizes sz;
  if ((st = validate(h, P, &sz, true))) return st;
  if (!plan || !plan->col_off || !plan->colmap || !plan->colscale) return fail(h, SBMM_E_ARG, "plan buffers missing");
  if (P->in_dtype != SBMM_F32) return fail(h, SBMM_E_UNSUPPORTED, "the MX E4M3 sketch takes float32 inputs");
  const int64_t nsc = round_up(sz.L_pad_max / 32, 4);
  if (C && (!Cs || ldc < sz.L_pad_max || ldc % 16 || ldcs < nsc || ldcs % 4))
    return fail(h, SBMM_E_ARG, "C needs ldc >= L_pad_max (multiple of 16) and scales Cs with ldcs >= %lld (multiple of 4)",
                (long long)nsc);
  if (Dt && (!Ds || lddt < sz.L_pad_max || lddt % 16 || ldds < nsc || ldds % 4))
    return fail(h, SBMM_E_ARG, "Dt needs lddt >= L_pad_max (multiple of 16) and scales Ds with ldds >= %lld (multiple of 4)",
                (long long)nsc);
  if ((C && (uintptr_t)C % 16) || (Dt && (uintptr_t)Dt % 16) || (Cs && (uintptr_t)Cs % 4) || (Ds && (uintptr_t)Ds % 4))
    return fail(h, SBMM_E_ARG, "C / Dt must be 16-byte aligned, Cs / Ds 4-byte aligned");
  MxGatherLaunch g{};
  g.M = reinterpret_cast<const float*>(P->M); g.ldm = P->ldm;
  g.N = reinterpret_cast<const float*>(P->N); g.ldn = P->ldn; g.m = P->m; g.p = P->p;
  g.L_dev = plan->col_off + P->c; g.L_pad_max = sz.L_pad_max;
  g.colmap = plan->colmap; g.colscale = plan->colscale;
  g.C = reinterpret_cast<uint8_t*>(C); g.ldc = ldc; g.Cs = reinterpret_cast<uint8_t*>(Cs); g.ldcs = ldcs;
  g.Dt = reinterpret_cast<uint8_t*>(Dt); g.lddt = lddt; g.Ds = reinterpret_cast<uint8_t*>(Ds); g.ldds = ldds;
  HIP_TRY(h, launch_mx_gather(g, (hipStream_t)stream));
  return SBMM_OK;
}

sbmm_status sbmm_sketch_gemm_mx(sbmm_handle h, int64_t m, int64_t p, int64_t L_pad_max, const int64_t* L_dev,
                                const void* C, int64_t ldc, const void* Cs, int64_t ldcs, const void* Dt,
                                int64_t lddt, const void* Ds, int64_t ldds, float* CD, int64_t ldcd,
                                const float* MN, int64_t ldmn, double* err_sq, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  if (m < 0 || p < 0 || L_pad_max < 0 || !L_dev) return fail(h, SBMM_E_ARG, "bad sizes or L_dev");
  const int64_t nsc = round_up(L_pad_max / 32, 4);
  if (m > 0 && p > 0 && L_pad_max > 0) {
    if (!C || !Cs || !Dt || !Ds) return fail(h, SBMM_E_ARG, "C, Cs, Dt and Ds are required");
    if (ldc < L_pad_max || ldc % 16 || lddt < L_pad_max || lddt % 16 || ldcs < nsc || ldcs % 4 || ldds < nsc ||
        ldds % 4)
      return fail(h, SBMM_E_ARG, "leading dimensions: ldc, lddt >= L_pad_max (multiples of 16); ldcs, ldds >= %lld "
                  "(multiples of 4)", (long long)nsc);
    if ((uintptr_t)C % 16 || (uintptr_t)Dt % 16 || (uintptr_t)Cs % 4 || (uintptr_t)Ds % 4)
      return fail(h, SBMM_E_ARG, "C / Dt must be 16-byte aligned, Cs / Ds 4-byte aligned");
  }
  if (CD && ldcd < p) return fail(h, SBMM_E_ARG, "ldcd < p");
  if ((MN != nullptr) != (err_sq != nullptr)) return fail(h, SBMM_E_ARG, "MN and err_sq go together");
  if (MN && ldmn < p) return fail(h, SBMM_E_ARG, "ldmn < p");
  hipStream_t s = (hipStream_t)stream;
  const int64_t tiles = mx_gemm_tiles(m, p);
  if ((st = ensure_ws(h, 512 + sizeof(double) * 2 * std::max<int64_t>(tiles, 1)))) return st;
  Arena ar(h->ws);
  double* tile_part = ar.take<double>(2 * std::max<int64_t>(tiles, 1));
  if (tiles == 0) {
    if (err_sq) HIP_TRY(h, launch_fill_f64(err_sq, 1, 0.0, s));
    return SBMM_OK;
  }
  MxGemmLaunch G{};
  G.A = reinterpret_cast<const uint8_t*>(C); G.lda = ldc; G.As = reinterpret_cast<const uint8_t*>(Cs); G.ldas = ldcs;
  G.B = reinterpret_cast<const uint8_t*>(Dt); G.ldb = lddt; G.Bs = reinterpret_cast<const uint8_t*>(Ds); G.ldbs = ldds;
  G.m = m; G.p = p; G.K_dev = L_dev; G.Cout = CD; G.ldc = ldcd; G.Y = MN; G.ldy = ldmn;
  G.tile_part = err_sq ? tile_part : nullptr;
  HIP_TRY(h, launch_mx_gemm(G, s));
  if (err_sq) {
    // the squared-error partials (row 0 of tile_part) summed straight into
    // err_sq: one small kernel, no device-to-device copy behind it
    HIP_TRY(h, launch_reduce_cols(tile_part, 1, tiles, err_sq, s));
  }
  return SBMM_OK;
}

sbmm_status sbmm_peak_probe(sbmm_handle h, sbmm_dtype dtype, double* tflops) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  if (!tflops) return fail(h, SBMM_E_ARG, "tflops is NULL");
  const int dt = enum_raw(dtype);
  if (dt != SBMM_F32 && dt != SBMM_BF16 && dt != SBMM_F8E4M3)
    return fail(h, SBMM_E_UNSUPPORTED, "no matrix-core probe for dtype %d", dt);
  HIP_TRY(h, hipSetDevice(h->device));
  int cus = 0;
  HIP_TRY(h, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, h->device));
  const int grid = 4 * std::max(cus, 1);
  // about 5-10 ms per launch at these instructions' rates
  const int64_t iters = dt == SBMM_BF16 ? 16384 : 8192;
  if ((st = ensure_ws(h, sizeof(float) * (size_t)grid * 256))) return st;
  float* out = reinterpret_cast<float*>(h->ws);
  struct Events {   // destroyed on every return path
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  HIP_TRY(h, hipEventCreate(&ev.a));
  HIP_TRY(h, hipEventCreate(&ev.b));
  int64_t count = 0;
  HIP_TRY(h, launch_mfma_peak(dtype, grid, iters, out, &count, nullptr));   // warm-up (clock ramp)
  HIP_TRY(h, hipEventRecord(ev.a, nullptr));
  HIP_TRY(h, launch_mfma_peak(dtype, grid, iters, out, &count, nullptr));
  HIP_TRY(h, hipEventRecord(ev.b, nullptr));
  HIP_TRY(h, hipEventSynchronize(ev.b));
  float ms = 0.0f;
  HIP_TRY(h, hipEventElapsedTime(&ms, ev.a, ev.b));
  *tflops = ms > 0.0f ? (double)count * (double)mfma_peak_flops_per_instruction(dtype) / ((double)ms * 1e9) : 0.0;
  return SBMM_OK;
}

sbmm_status sbmm_error(sbmm_handle h, int64_t m, int64_t p, sbmm_dtype dtype, const void* X, int64_t ldx,
                       const void* Y, int64_t ldy, double* out2, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  if (m < 0 || p < 0 || !out2) return fail(h, SBMM_E_ARG, "bad sizes or out2");
  if (enum_raw(dtype) != SBMM_F64 && enum_raw(dtype) != SBMM_F32) return fail(h, SBMM_E_ARG, "dtype must be F64 or F32");
  if (m > 0 && p > 0 && (!X || !Y || ldx < p || ldy < p)) return fail(h, SBMM_E_ARG, "X/Y missing or ld < p");
  hipStream_t s = (hipStream_t)stream;
  if (m == 0 || p == 0) {
    HIP_TRY(h, launch_fill_f64(out2, 2, 0.0, s));
    return SBMM_OK;
  }
  const int64_t np = error_parts(m, p);
  if ((st = ensure_ws(h, 256 + sizeof(double) * 2 * np))) return st;
  Arena ar(h->ws);
  double* part = ar.take<double>(2 * np);
  HIP_TRY(h, launch_error(dtype, m, p, X, ldx, Y, ldy, part, np, s));
  HIP_TRY(h, launch_reduce_cols(part, 2, np, out2, s));
  return SBMM_OK;
}

}  // extern "C"

namespace {

// The whole forward path. With `measure` non-null nothing is launched or
// allocated (h may then be null): *measure receives the workspace bytes the
// call needs, from the same arena layout as the real pass.
sbmm_status run_impl(sbmm_handle h, const sbmm_problem* P, sbmm_dtype compute, void* C, int64_t ldc, void* D,
                     int64_t ldd, void* CD, int64_t ldcd, void* MN, int64_t ldmn, const sbmm_plan_out* plan,
                     double* err_host, double* rel_host, int64_t* L_host, sbmm_stream stream, size_t* measure) {
  sbmm_status st = SBMM_OK;
  sbmm_sizes sz;
  if ((st = validate(h, P, &sz, true))) return st;
  if (!plan_out_ok(plan)) return fail(h, SBMM_E_ARG, "plan output buffers missing");
  if (!sketch_dtype_ok(P->in_dtype, compute)) return fail(h, SBMM_E_ARG, "compute dtype not allowed for the input dtype");
  if (enum_raw(compute) != SBMM_F64 && enum_raw(compute) != SBMM_F32 && enum_raw(compute) != SBMM_BF16)
    return fail(h, SBMM_E_UNSUPPORTED, "sketched product in dtype %d is not built", enum_raw(compute));
  if ((P->m > 0 && P->p > 0 && !CD) || ldcd < P->p) return fail(h, SBMM_E_ARG, "CD is required with ldcd >= p");
  if (C && ldc < sz.L_pad_max) return fail(h, SBMM_E_ARG, "ldc < L_pad_max");
  if (D && ldd < P->p) return fail(h, SBMM_E_ARG, "ldd < p");
  if (MN && ldmn < P->p) return fail(h, SBMM_E_ARG, "ldmn < p");
  const bool two = P->mode == SBMM_MODE_STRATIFIED && P->alloc == SBMM_ALLOC_TWO_STEP;
  if (two && (st = validate_pilot(h, P))) return st;
  hipStream_t s = (hipStream_t)stream;
  const bool bp = needs_blkprod(P);
  const bool own_pilot = two && !P->pilot_sq;
  const sbmm_dtype pd = product_dtype(P->in_dtype);
  const size_t pes = dtype_size(pd), ces = dtype_size(compute);

  for (int pass = 0; pass < 2; ++pass) {
    Arena ar(pass ? h->ws : nullptr);
    int64_t* off = nullptr;
    if ((st = upload_offsets(h, P, ar, &off, s))) return st;
    double* col_sq = ar.take<double>(P->n);
    double* row_sq = ar.take<double>(P->n);
    double* blk = ar.take<double>(3 * (size_t)P->K);
    double* blkprod = bp ? ar.take<double>(P->K) : nullptr;
    double* pilot = own_pilot ? ar.take<double>(P->K) : nullptr;
    double* ex2 = ar.take<double>(2);     // exact pass: err^2 (when fused), ||MN||^2
    double* sk2 = ar.take<double>(2);     // sketch pass: err^2, ||CD||^2
    void* Cw = C ? C : ar.take<char>(ces * (size_t)std::max<int64_t>(P->m, 1) * sz.L_pad_max);
    const int64_t ldcw = C ? ldc : sz.L_pad_max;
    void* Dw = D ? D : ar.take<char>(ces * (size_t)sz.L_pad_max * std::max<int64_t>(P->p, 1));
    const int64_t lddw = D ? ldd : P->p;
    void* MNw = MN ? MN : (bp ? ar.take<char>(pes * (size_t)std::max<int64_t>(P->m, 1) * std::max<int64_t>(P->p, 1)) : nullptr);
    const int64_t ldmnw = MN ? ldmn : P->p;
    GemmLaunch Gs{};   // the sketched product (step 5)
    Gs.dt = compute; Gs.A = Cw; Gs.lda = ldcw; Gs.B = Dw; Gs.ldb = lddw; Gs.m = P->m; Gs.p = P->p;
    Gs.K_host = 0; Gs.K_dev = plan->col_off + P->c; Gs.K_max = sz.L_pad_max;
    const int64_t tiles_s = compute == SBMM_BF16 ? hgemm_tiles(Gs) : gemm_tiles(compute, P->m, P->p, false);
    double* sk_part = ar.take<double>(2 * std::max<int64_t>(tiles_s, 1));
    float* sk_stage = ar.take<float>(gemm_stage_bytes(compute, P->m, P->p) / sizeof(float));
    const size_t skb = compute == SBMM_BF16 ? 0 : gemm_skinny_ws_bytes(compute, P->m, P->p, sz.L_pad_max, 0);
    void* sk_skinny = skb ? ar.take<char>(skb) : nullptr;
    // measure the remaining scratch of the sub-steps on a dry arena
    if (!pass) {
      do_norms(h, P, off, col_sq, row_sq, blk, ar, s);
      Arena sub(nullptr);
      sub.off = ar.off;
      do_exact(h, P, off, MNw, ldmnw, nullptr, 0, blkprod, ex2, sub, s);
      size_t need = sub.off;
      Arena sub2(nullptr);
      sub2.off = ar.off;
      do_plan(h, P, sz, off, col_sq, row_sq, blk, plan, sub2, s);
      need = std::max(need, sub2.off);
      if (own_pilot) {
        Arena sub3(nullptr);
        sub3.off = ar.off;
        do_pilot(h, P, off, col_sq, row_sq, blk, nullptr, pilot, sub3, s);
        need = std::max(need, sub3.off);
      }
      if (measure) {
        *measure = need;
        return SBMM_OK;
      }
      if ((st = ensure_ws(h, need))) return st;
      continue;
    }
    const size_t base = ar.off;
    // 1. norm pass
    {
      Arena sub(h->ws);
      sub.off = base;
      if ((st = do_norms(h, P, off, col_sq, row_sq, blk, sub, s))) return st;
    }
    // 2. exact product first when the rules need ||M^k N_k||_F
    if (bp) {
      Arena sub(h->ws);
      sub.off = base;
      if ((st = do_exact(h, P, off, MNw, ldmnw, nullptr, 0, blkprod, ex2, sub, s))) return st;
    }
    // 3. plan (after the pilot of the two-step algorithm, Alg. 3 step 1)
    sbmm_problem Q = *P;
    if (bp) Q.blkprod_sq = blkprod;
    if (own_pilot) {
      Arena sub(h->ws);
      sub.off = base;
      if ((st = do_pilot(h, P, off, col_sq, row_sq, blk, nullptr, pilot, sub, s))) return st;
      Q.pilot_sq = pilot;
    }
    {
      Arena sub(h->ws);
      sub.off = base;
      if ((st = do_plan(h, &Q, sz, off, col_sq, row_sq, blk, plan, sub, s))) return st;
    }
    // 4. sketch
    {
      GatherLaunch g{};
      g.in_dt = P->in_dtype; g.out_dt = compute;
      g.M = P->M; g.ldm = P->ldm; g.N = P->N; g.ldn = P->ldn; g.m = P->m; g.p = P->p;
      g.L_dev = plan->col_off + P->c; g.L_pad_max = sz.L_pad_max;
      g.colmap = plan->colmap; g.colscale = plan->colscale;
      g.C = Cw; g.ldc = ldcw; g.D = Dw; g.ldd = lddw;
      HIP_TRY(h, launch_gather(g, s));
    }
    // 5. sketched product (with the error when MN is already there)
    if (tiles_s > 0) {
      GemmLaunch G = Gs;
      G.Cout = CD; G.ldc = ldcd;
      G.Y = bp ? MNw : nullptr; G.ldy = ldmnw; G.tile_part = bp ? sk_part : nullptr;
      G.stage = sk_stage;
      G.skinny_ws = sk_skinny; G.skinny_K_max = sz.L_pad_max;
      HIP_TRY(h, run_product(G, s));
      if (bp) HIP_TRY(h, launch_reduce_cols(sk_part, 2, tiles_s, sk2, s));
    }
    // 6. exact product with the error against CD
    if (!bp) {
      Arena sub(h->ws);
      sub.off = base;
      if ((st = do_exact(h, P, off, MNw, ldmnw, CD, ldcd, nullptr, ex2, sub, s))) return st;
    }
    // 7. results
    double hv[4] = {0, 0, 0, 0};
    int64_t Lh = 0;
    HIP_TRY(h, hipMemcpyAsync(hv, ex2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    if (bp && tiles_s > 0) HIP_TRY(h, hipMemcpyAsync(hv + 2, sk2, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipMemcpyAsync(&Lh, plan->col_off + P->c, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    if ((st = read_status(h, s))) return st;
    const double err2 = bp ? hv[2] : hv[0];
    const double mn2 = hv[1];
    const double err = std::sqrt(err2);
    if (err_host) *err_host = err;
    if (rel_host) *rel_host = mn2 > 0 ? err / std::sqrt(mn2) : (err2 > 0 ? INFINITY : 0.0);
    if (L_host) *L_host = Lh;
  }
  return SBMM_OK;
}

}  // namespace

extern "C" {

sbmm_status sbmm_bound(sbmm_handle h, const sbmm_problem* P, const double* col_sq, const double* row_sq,
                       const double* blk, const double* blkprod_sq, const sbmm_plan_out* plan, double beta,
                       int32_t n_delta, const double* delta, double* out, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  if ((st = validate(h, P, nullptr, true))) return st;
  if (P->mode != SBMM_MODE_STRATIFIED) return fail(h, SBMM_E_ARG, "the bounds are those of the stratified sampler");
  if (P->alloc != SBMM_ALLOC_OPT && P->alloc != SBMM_ALLOC_NORM && P->alloc != SBMM_ALLOC_TWO_STEP)
    return fail(h, SBMM_E_ARG, "no bound for block-size rule %d (OPT, NORM or TWO_STEP)", (int)P->alloc);
  if (P->alloc == SBMM_ALLOC_TWO_STEP && !P->pilot_sq) return fail(h, SBMM_E_ARG, "TWO_STEP needs prob->pilot_sq");
  if (!col_sq || !row_sq || !blk || !blkprod_sq || !plan || !plan->p_hat || !plan->ck || !out)
    return fail(h, SBMM_E_ARG, "the bounds need col_sq, row_sq, blk, blkprod_sq, plan p_hat and ck, and out");
  if (n_delta < 0 || n_delta > SBMM_BOUND_MAX_DELTA || (n_delta > 0 && !delta))
    return fail(h, SBMM_E_ARG, "n_delta = %d (0..%d)", n_delta, (int)SBMM_BOUND_MAX_DELTA);
  if (!(beta >= 0.0 && beta <= 1.0)) return fail(h, SBMM_E_ARG, "beta must be in [0, 1]");
  BoundLaunch a{};
  for (int32_t j = 0; j < n_delta; ++j) {
    if (!(delta[j] > 0.0 && delta[j] < 1.0)) return fail(h, SBMM_E_ARG, "delta[%d] must be in (0, 1)", j);
    a.delta[j] = delta[j];
  }
  std::vector<int64_t> chunk_off(P->K + 1, 0);
  for (int32_t k = 0; k < P->K; ++k)
    chunk_off[k + 1] = chunk_off[k] + bound_chunks(P->block_off[k + 1] - P->block_off[k]);
  const int64_t nout = SBMM_BOUND_FIXED + 2 * (int64_t)n_delta;
  hipStream_t s = (hipStream_t)stream;
  for (int pass = 0; pass < 2; ++pass) {
    Arena ar(pass ? h->ws : nullptr);
    int64_t* off = nullptr;
    if ((st = upload_offsets(h, P, ar, &off, s))) return st;
    int64_t* coff = ar.take<int64_t>(P->K + 1);
    double* part = ar.take<double>(2 * (size_t)chunk_off[P->K]);
    double* dout = ar.take<double>(nout);
    if (!pass) {
      if ((st = ensure_ws(h, ar.off))) return st;
      continue;
    }
    HIP_TRY(h, hipMemcpyAsync(coff, chunk_off.data(), sizeof(int64_t) * (P->K + 1), hipMemcpyHostToDevice, s));
    a.K = P->K; a.off = off; a.chunk_off = coff; a.chunks = chunk_off[P->K];
    a.col_sq = col_sq; a.row_sq = row_sq; a.blk = blk; a.blkprod_sq = blkprod_sq;
    a.pilot_sq = P->alloc == SBMM_ALLOC_TWO_STEP ? P->pilot_sq : nullptr;
    a.p_hat = plan->p_hat; a.ck = plan->ck; a.part = part;
    a.rule = P->alloc; a.c = P->c; a.beta = beta; a.n_delta = n_delta; a.out = dout;
    HIP_TRY(h, launch_bound(a, s));
    HIP_TRY(h, hipMemcpyAsync(out, dout, sizeof(double) * nout, hipMemcpyDeviceToHost, s));
    HIP_TRY(h, hipStreamSynchronize(s));
  }
  return SBMM_OK;
}

sbmm_status sbmm_run(sbmm_handle h, const sbmm_problem* P, sbmm_dtype compute, void* C, int64_t ldc, void* D,
                     int64_t ldd, void* CD, int64_t ldcd, void* MN, int64_t ldmn, const sbmm_plan_out* plan,
                     double* err_host, double* rel_host, int64_t* L_host, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  return run_impl(h, P, compute, C, ldc, D, ldd, CD, ldcd, MN, ldmn, plan, err_host, rel_host, L_host, stream,
                  nullptr);
}

sbmm_status sbmm_exact_error(sbmm_handle h, const sbmm_problem* P, const void* CD, int64_t ldcd,
                             sbmm_dtype cd_dtype, void* MN, int64_t ldmn, double* blkprod_sq,
                             double* err2_and_mn2, sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  sbmm_sizes sz;
  if ((st = validate(h, P, &sz, true))) return st;
  if (!err2_and_mn2) return fail(h, SBMM_E_ARG, "err2_and_mn2 is required");
  if (enum_raw(cd_dtype) != (int)product_dtype(P->in_dtype))
    return fail(h, SBMM_E_ARG, "CD must be in the product dtype (F64 for F64 inputs, else F32)");
  if ((P->m > 0 && P->p > 0 && !CD) || ldcd < P->p) return fail(h, SBMM_E_ARG, "CD is required with ldcd >= p");
  if (MN && ldmn < P->p) return fail(h, SBMM_E_ARG, "ldmn < p");
  hipStream_t s = (hipStream_t)stream;
  Arena dry(nullptr);
  int64_t* off = nullptr;
  upload_offsets(h, P, dry, &off, s);
  if ((st = do_exact(h, P, off, MN, ldmn, CD, ldcd, blkprod_sq, err2_and_mn2, dry, s))) return st;
  if ((st = ensure_ws(h, dry.off))) return st;
  Arena ar(h->ws);
  if ((st = upload_offsets(h, P, ar, &off, s))) return st;
  return do_exact(h, P, off, MN, ldmn, CD, ldcd, blkprod_sq, err2_and_mn2, ar, s);
}

sbmm_status sbmm_workspace_size(const sbmm_problem* P, sbmm_dtype compute, size_t* bytes, int64_t* L_max) {
  if (!bytes) return SBMM_E_ARG;
  sbmm_sizes sz;
  sbmm_status st = validate(nullptr, P, &sz, true);
  if (st) return st;
  if (!sketch_dtype_ok(P->in_dtype, compute)) return SBMM_E_ARG;
  // placeholders: never dereferenced by a measuring pass
  char* const ph = reinterpret_cast<char*>((uintptr_t)256);
  sbmm_plan_out pl{};
  pl.idx = reinterpret_cast<int32_t*>(ph); pl.scale = reinterpret_cast<double*>(ph);
  pl.col_off = reinterpret_cast<int64_t*>(ph); pl.ck = reinterpret_cast<int64_t*>(ph);
  pl.colmap = reinterpret_cast<int32_t*>(ph); pl.colscale = reinterpret_cast<double*>(ph);
  size_t need = 0, x = 0;
  // sbmm_run with C, D and MN left to the library
  if ((st = run_impl(nullptr, P, compute, nullptr, 0, nullptr, 0, ph, P->p, nullptr, 0, &pl, nullptr, nullptr,
                     nullptr, nullptr, &x)))
    return st;
  need = std::max(need, x);
  int64_t* off = nullptr;
  // sbmm_exact / sbmm_exact_error with per-block norms
  if (P->in_dtype != SBMM_BF16) {
    Arena dry(nullptr);
    upload_offsets(nullptr, P, dry, &off, nullptr);
    double* out2 = dry.take<double>(2);
    if ((st = do_exact(nullptr, P, off, nullptr, 0, nullptr, 0, reinterpret_cast<double*>(ph), out2, dry, nullptr)))
      return st;
    need = std::max(need, dry.off);
  }
  // sbmm_pilot without a pilot plan of the caller's
  if (P->mode == SBMM_MODE_STRATIFIED && P->alloc == SBMM_ALLOC_TWO_STEP) {
    if ((st = validate_pilot(nullptr, P))) return st;
    Arena dry(nullptr);
    upload_offsets(nullptr, P, dry, &off, nullptr);
    do_pilot(nullptr, P, off, nullptr, nullptr, nullptr, nullptr, reinterpret_cast<double*>(ph), dry, nullptr);
    need = std::max(need, dry.off);
  }
  // sbmm_bound with eight deltas
  if (P->mode == SBMM_MODE_STRATIFIED) {
    int64_t chunks = 0;
    for (int32_t k = 0; k < P->K; ++k) chunks += bound_chunks(P->block_off[k + 1] - P->block_off[k]);
    Arena dry(nullptr);
    dry.take<int64_t>(P->K + 1);
    dry.take<double>(2 * (size_t)chunks);
    dry.take<double>(SBMM_BOUND_FIXED + 2 * SBMM_BOUND_MAX_DELTA);
    need = std::max(need, dry.off);
  }
  *bytes = need;
  if (L_max) *L_max = sz.L_max;
  return SBMM_OK;
}

sbmm_status sbmm_backward(sbmm_handle h, const sbmm_problem* P, const sbmm_plan_out* plan, int64_t L,
                          sbmm_dtype compute, const void* C, int64_t ldc, const void* D, int64_t ldd,
                          const void* G, int64_t ldg, void* dM, int64_t lddm, void* dN, int64_t lddn,
                          sbmm_stream stream) {
  sbmm_status st = check_handle(h);
  if (st) return st;
  sbmm_sizes sz;
  if ((st = validate(h, P, &sz, true))) return st;
  if (!plan || !plan->idx || !plan->scale || !plan->col_off) return fail(h, SBMM_E_ARG, "plan buffers missing");
  if (!sketch_dtype_ok(P->in_dtype, compute)) return fail(h, SBMM_E_ARG, "compute dtype not allowed for the input dtype");
  if (L < 0 || L > sz.L_pad_max) return fail(h, SBMM_E_ARG, "L must lie in [0, L_pad_max]");
  const int64_t m = P->m, n = P->n, p = P->p;
  if ((m > 0 && !dM) || (p > 0 && !dN)) return fail(h, SBMM_E_ARG, "dM and dN are required");
  if ((dM && lddm < n) || (dN && lddn < p)) return fail(h, SBMM_E_ARG, "lddm < n or lddn < p");
  // bf16: the draws merged per atom, both products over the compact width
  // with their epilogues writing dM / dN (operands padded to whole 16-byte
  // chunks; the 256 x 256 kernel's panels need 32-bit offsets). This form
  // reads M and N, not C and D.
  const int64_t ldp8 = round_up(std::max<int64_t>(p, 1), 8), ldm8 = round_up(std::max<int64_t>(m, 1), 8);
  const bool merged = compute == SBMM_BF16 && 257 * std::max(ldp8, ldm8) * 2 < ((int64_t)1 << 31);
  if (L > 0 && m > 0 && p > 0) {
    if (!G || (!merged && (!C || !D))) return fail(h, SBMM_E_ARG, "C, D and G are required");
    if (ldg < p || (!merged && (ldc < L || ldd < p))) return fail(h, SBMM_E_ARG, "ldc < L, ldd < p or ldg < p");
  }
  hipStream_t s = (hipStream_t)stream;
  const sbmm_dtype gd = compute == SBMM_F64 ? SBMM_F64 : SBMM_F32;   // dtype of G, dC, dD
  const size_t ges = dtype_size(gd);
  if (merged && L > 0 && m > 0 && p > 0) {
    const int64_t Lu = std::min<int64_t>(L, n);   // compact width bound
    for (int pass = 0; pass < 2; ++pass) {
      Arena ar(pass ? h->ws : nullptr);
      int64_t* off = nullptr;
      if ((st = upload_offsets(h, P, ar, &off, s))) return st;
      int32_t* cnt = ar.take<int32_t>(sz.atoms);
      int32_t* rank = ar.take<int32_t>(P->c);
      int64_t* aoff = ar.take<int64_t>(sz.atoms + 1);
      int32_t* list = ar.take<int32_t>(P->c);
      BackwardDedup d{};
      d.uoff = ar.take<int64_t>(sz.atoms);
      d.wsum = ar.take<double>(sz.atoms);
      d.ucol = ar.take<int32_t>(Lu);
      d.uw = ar.take<double>(Lu);
      d.drawn = ar.take<uint8_t>(n);
      d.lu = ar.take<int64_t>(1);
      uint16_t* NU = ar.take<uint16_t>((size_t)Lu * ldp8);
      uint16_t* MUt = ar.take<uint16_t>((size_t)Lu * ldm8);
      uint16_t* G16 = ar.take<uint16_t>((size_t)m * ldp8);
      uint16_t* G16t = ar.take<uint16_t>((size_t)p * ldm8);
      if (!pass) {
        if ((st = ensure_ws(h, ar.off))) return st;
        continue;
      }
      HIP_TRY(h, launch_draw_lists(plan->idx, P->c, sz.atoms, cnt, rank, aoff, list, s));
      d.mode = P->mode; d.off_dev = off; d.K = P->K; d.A = sz.atoms; d.n = n;
      d.cnt = cnt; d.aoff = aoff; d.list = list; d.scale = plan->scale; d.cap = Lu; d.status = h->status;
      HIP_TRY(h, launch_dedup(d, s));
      HIP_TRY(h, launch_g_prep(reinterpret_cast<const float*>(G), ldg, m, p, G16, ldp8, G16t, ldm8, s));
      HIP_TRY(h, launch_gather_compact(P->in_dtype, P->N, P->ldn, p, P->M, P->ldm, m, d.ucol, d.lu, Lu, NU, ldp8,
                                       MUt, ldm8, s));
      HIP_TRY(h, launch_zero_undrawn(P->in_dtype, dM, lddm, m, dN, lddn, p, n, d.drawn, s));
      GemmLaunch g1{};   // dM[:, ucol] = uw * (G N_U^T)   (m x Lu, inner p)
      g1.dt = SBMM_BF16; g1.A = G16; g1.lda = ldp8; g1.B = NU; g1.ldb = ldp8; g1.b_trans = true;
      g1.m = m; g1.p = Lu; g1.p_dev = d.lu; g1.K_host = ldp8;
      g1.sc_mode = SC_COLS; g1.sc_out = dM; g1.sc_ld = lddm; g1.sc_f32 = P->in_dtype == SBMM_F32;
      g1.sc_map = d.ucol; g1.sc_w = d.uw;
      HIP_TRY(h, launch_gemm(g1, s));
      GemmLaunch g2{};   // dN[ucol, :] = uw * (M_U^T G)   (Lu x p, inner m)
      g2.dt = SBMM_BF16; g2.A = MUt; g2.lda = ldm8; g2.B = G16t; g2.ldb = ldm8; g2.b_trans = true;
      g2.m = Lu; g2.m_dev = d.lu; g2.p = p; g2.K_host = ldm8;
      g2.sc_mode = SC_ROWS; g2.sc_out = dN; g2.sc_ld = lddn; g2.sc_f32 = P->in_dtype == SBMM_F32;
      g2.sc_map = d.ucol; g2.sc_w = d.uw;
      HIP_TRY(h, launch_gemm(g2, s));
    }
    return SBMM_OK;
  }
  for (int pass = 0; pass < 2; ++pass) {
    Arena ar(pass ? h->ws : nullptr);
    int64_t* off = nullptr;
    if ((st = upload_offsets(h, P, ar, &off, s))) return st;
    int32_t* cnt = ar.take<int32_t>(sz.atoms);
    int32_t* rank = ar.take<int32_t>(P->c);
    int64_t* aoff = ar.take<int64_t>(sz.atoms + 1);
    int32_t* list = ar.take<int32_t>(P->c);
    char* dC = ar.take<char>(ges * (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(L, 1));
    char* dD = ar.take<char>(ges * (size_t)std::max<int64_t>(L, 1) * std::max<int64_t>(p, 1));
    const bool bf = compute == SBMM_BF16;
    const size_t mp = (size_t)std::max<int64_t>(m, 1) * std::max<int64_t>(p, 1);
    uint16_t* G16 = bf ? ar.take<uint16_t>(mp) : nullptr;                 // G, m x p
    uint16_t* G16t = bf ? ar.take<uint16_t>(mp) : nullptr;                // G^T, p x m
    uint16_t* Ct = bf ? ar.take<uint16_t>((size_t)std::max<int64_t>(L, 1) * std::max<int64_t>(m, 1)) : nullptr;  // C^T, L x m
    if (!pass) {
      if ((st = ensure_ws(h, ar.off))) return st;
      continue;
    }
    HIP_TRY(h, launch_draw_lists(plan->idx, P->c, sz.atoms, cnt, rank, aoff, list, s));
    if (L > 0 && m > 0 && p > 0) {
      if (compute == SBMM_BF16) {
        HIP_TRY(h, launch_to_bf16(reinterpret_cast<const float*>(G), m, p, ldg, G16, s));
        GemmLaunch g1{};   // dC = G D^T  (m x L, inner p)
        g1.dt = SBMM_BF16; g1.A = G16; g1.lda = p; g1.B = D; g1.ldb = ldd; g1.b_trans = true;
        g1.m = m; g1.p = L; g1.K_host = p; g1.Cout = dC; g1.ldc = L;
        HIP_TRY(h, launch_gemm(g1, s));
        // dD = C^T G  (L x p, inner m) from C^T (L x m) and G^T (p x m)
        HIP_TRY(h, launch_transpose_bf16(SBMM_F32, G, m, p, ldg, nullptr, G16t, m, s));
        HIP_TRY(h, launch_transpose_bf16(SBMM_BF16, C, m, L, ldc, nullptr, Ct, m, s));
        GemmLaunch g2{};
        g2.dt = SBMM_BF16; g2.A = Ct; g2.lda = m; g2.B = G16t; g2.ldb = m; g2.b_trans = true;
        g2.m = L; g2.p = p; g2.K_host = m; g2.Cout = dD; g2.ldc = p;
        HIP_TRY(h, launch_gemm(g2, s));
      } else {
        HIP_TRY(h, launch_gemm_strided(gd, G, ldg, 1, D, 1, ldd, dC, L, m, L, p, s));
        HIP_TRY(h, launch_gemm_strided(gd, C, 1, ldc, G, ldg, 1, dD, p, L, p, m, s));
      }
    } else {
      if (m > 0 && L > 0) HIP_TRY(h, launch_fill_f64(reinterpret_cast<double*>(dC), (int64_t)(ges * m * L / 8), 0.0, s));
      if (p > 0 && L > 0) HIP_TRY(h, launch_fill_f64(reinterpret_cast<double*>(dD), (int64_t)(ges * L * p / 8), 0.0, s));
    }
    BackwardScatter b{};
    b.mode = P->mode; b.off_dev = off; b.K = P->K; b.aoff = aoff; b.list = list;
    b.scale = plan->scale; b.col_off = plan->col_off; b.m = m; b.n = n; b.p = p;
    b.grad_dt = gd; b.out_dt = P->in_dtype; b.dC = dC; b.lddc = std::max<int64_t>(L, 1);
    b.dD = dD; b.lddd = std::max<int64_t>(p, 1); b.dM = dM; b.lddm = lddm; b.dN = dN; b.lddn = lddn;
    b.L = L; b.status = h->status;
    HIP_TRY(h, launch_scatter(b, s));
  }
  return SBMM_OK;
}

}  // extern "C"
