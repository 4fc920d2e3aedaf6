// Host side of libtacsl: scene validation, work-list construction, plans,
// the extern "C" entry points of include/tacsl.h, and substep graphs.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "tacsl.h"
#include "tacsl_internal.h"

using tacsl::InstStatic;
using tacsl::InstXf;
using tacsl::Tile;

namespace {

// Host-side range around each entry point that enqueues device work, named
// after it; rocprofv3 --marker-trace shows them (a no-op with no tool attached).
struct Range {
  explicit Range(const char* name) { roctxRangePushA(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

constexpr int64_t kMaxGridBytes = (int64_t(1) << 32) - 1;  // prepared grid addressed with 32-bit offsets
constexpr int64_t kMaxPairStride = (int64_t(1) << 24) - 1;  // bytes per x-pair: a 24-bit multiplier operand
constexpr int64_t kMaxTemplate = int64_t(1) << 30;
constexpr int kXcdCount = 8;  // MI355X: 8 XCDs, workgroups dispatched round-robin across them

int64_t tmpl_count(const tacsl_scene_desc& d, int i) {
  const int p = d.inst_tmpl[i];
  return d.tmpl_offset[p + 1] - d.tmpl_offset[p];
}

int validate(const tacsl_scene_desc* d) {
  if (!d) return TACSL_ERR_NULL_ARG;
  if (d->n_env < 0 || d->n_inst < 0 || d->n_tmpl < 0 || d->n_sdf < 0) return TACSL_ERR_SHAPE;
  if (d->n_inst > 0 && (d->n_env < 1 || d->n_tmpl < 1 || d->n_sdf < 1)) return TACSL_ERR_SHAPE;
  if (d->n_inst > 0 && (!d->inst_env || !d->inst_tmpl)) return TACSL_ERR_NULL_ARG;
  if (d->n_env > 0 && !d->env_sdf) return TACSL_ERR_NULL_ARG;
  if (d->n_tmpl > 0 && !d->tmpl_offset) return TACSL_ERR_NULL_ARG;
  if (d->n_sdf > 0 && (!d->sdf_dims || !d->sdf_origin || !d->sdf_spacing || !d->sdf_offset || !d->sdf_data))
    return TACSL_ERR_NULL_ARG;
  if (d->n_tmpl > 0) {
    if (d->tmpl_offset[0] != 0) return TACSL_ERR_SHAPE;
    for (int p = 0; p < d->n_tmpl; ++p) {
      const int64_t c = d->tmpl_offset[p + 1] - d->tmpl_offset[p];
      if (c < 0) return TACSL_ERR_SHAPE;
      if (c > kMaxTemplate) return TACSL_ERR_UNSUPPORTED;
    }
    if (d->tmpl_offset[d->n_tmpl] > 0 && !d->tmpl_xyz) return TACSL_ERR_NULL_ARG;
  }
  for (int e = 0; e < d->n_env; ++e)
    if (d->env_sdf[e] < 0 || d->env_sdf[e] >= d->n_sdf) return TACSL_ERR_RANGE;
  for (int i = 0; i < d->n_inst; ++i) {
    if (d->inst_env[i] < 0 || d->inst_env[i] >= d->n_env) return TACSL_ERR_RANGE;
    if (d->inst_tmpl[i] < 0 || d->inst_tmpl[i] >= d->n_tmpl) return TACSL_ERR_RANGE;
  }
  for (int g = 0; g < d->n_sdf; ++g) {
    const int32_t* n = d->sdf_dims + 3 * g;
    if (n[0] < 2 || n[1] < 2 || n[2] < 2) return TACSL_ERR_SHAPE;
    if (tacsl::prepared_grid_bytes(n[0], n[1], n[2]) > kMaxGridBytes) return TACSL_ERR_UNSUPPORTED;
    if (int64_t(64) * ((n[1] + 1) / 2) * n[2] > kMaxPairStride) return TACSL_ERR_UNSUPPORTED;
    const float h = d->sdf_spacing[g];
    if (!(h > 0.f) || !std::isfinite(h)) return TACSL_ERR_RANGE;
    for (int a = 0; a < 3; ++a)
      if (!std::isfinite(d->sdf_origin[3 * g + a])) return TACSL_ERR_RANGE;
    if (d->sdf_offset[g] < 0) return TACSL_ERR_RANGE;
  }
  int64_t T = 0;
  for (int i = 0; i < d->n_inst; ++i) {
    T += tmpl_count(*d, i);
    if (T > (int64_t(1) << 40)) return TACSL_ERR_UNSUPPORTED;
  }
  return TACSL_OK;
}

int resolve_tuning(const tacsl_tuning* in, int cu_count, tacsl_tuning* out) {
  tacsl_tuning t = {0, 0, 0, 0, 0};
  if (in) t = *in;
  if (t.block == 0) t.block = 256;
  if (t.block != 64 && t.block != 128 && t.block != 256 && t.block != 512) return TACSL_ERR_RANGE;
  if (t.tile_taxels < 0 || (t.tile_taxels > 0 && t.tile_taxels < 64) || t.tile_taxels > kMaxTemplate)
    return TACSL_ERR_RANGE;
  if (t.schedule < 0 || t.schedule > 2) return TACSL_ERR_RANGE;
  if (t.order < 0 || t.order > 5) return TACSL_ERR_RANGE;
  if (t.grid < 0) return TACSL_ERR_RANGE;
  if (t.grid == 0) t.grid = std::max(1, cu_count) * 8;
  *out = t;
  return TACSL_OK;
}

// Tiles are numbered instance-major (every pad has >= 1 tile); `order` maps
// execution slots to tile ids.
int make_worklist(const tacsl_scene_desc& d, const tacsl_tuning& t, int xcd, std::vector<Tile>& tiles,
                  std::vector<int32_t>& order, std::vector<int64_t>& inst_tile_begin) {
  tiles.clear();
  order.clear();
  inst_tile_begin.assign((size_t)d.n_inst + 1, 0);
  for (int i = 0; i < d.n_inst; ++i) {
    inst_tile_begin[i] = (int64_t)tiles.size();
    const int64_t cnt = tmpl_count(d, i);
    if (cnt == 0) {
      tiles.push_back(Tile{i, 0, 0, d.inst_env[i]});
      continue;
    }
    const int64_t tsz = t.tile_taxels > 0 ? t.tile_taxels : cnt;
    for (int64_t k0 = 0; k0 < cnt; k0 += tsz)
      tiles.push_back(Tile{i, (int32_t)k0, (int32_t)std::min(tsz, cnt - k0), d.inst_env[i]});
    if ((int64_t)tiles.size() > (int64_t)INT32_MAX) return TACSL_ERR_UNSUPPORTED;
  }
  inst_tile_begin[d.n_inst] = (int64_t)tiles.size();
  const int32_t n = (int32_t)tiles.size();
  order.resize(n);
  std::iota(order.begin(), order.end(), 0);
  auto cost = [&](int32_t tid) { return (int64_t)std::max(tiles[tid].count, 1); };
  if (t.order == 2) {
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
  } else if (t.order == 3) {
    // object-major: all XCDs work on one object grid at a time
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return d.env_sdf[d.inst_env[tiles[a].inst]] < d.env_sdf[d.inst_env[tiles[b].inst]];
    });
  } else if ((t.order == 1 || t.order == 4 || t.order == 5) && n > 0) {
    // group by object grid.  Order 1: cut the whole list into xcd contiguous
    // segments of equal cost, interleaved so that slot s runs on XCD s % xcd
    // while segments last.  Order 4: the same per object grid, one object
    // after the other (object-major for the memory-side cache, and each XCD
    // on a contiguous run of the object's pads for its own L2).  Order 5
    // starts from order 4 and is rebuilt on the device every call with the
    // pads in spatial order.
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
      return d.env_sdf[d.inst_env[tiles[a].inst]] < d.env_sdf[d.inst_env[tiles[b].inst]];
    });
    auto interleave = [&](const std::vector<int32_t>& part, std::vector<int32_t>& dst) {
      int64_t total = 0;
      for (int32_t tid : part) total += cost(tid);
      std::vector<std::vector<int32_t>> seg((size_t)xcd);
      int64_t acc = 0;
      int x = 0;
      for (int32_t tid : part) {
        while (x < xcd - 1 && acc >= (total * (x + 1)) / xcd) ++x;
        seg[x].push_back(tid);
        acc += cost(tid);
      }
      std::vector<size_t> pos((size_t)xcd, 0);
      bool more = true;
      while (more) {
        more = false;
        for (int s2 = 0; s2 < xcd; ++s2)
          if (pos[s2] < seg[s2].size()) {
            dst.push_back(seg[s2][pos[s2]++]);
            more = true;
          }
      }
    };
    std::vector<int32_t> out;
    out.reserve(order.size());
    if (t.order == 1) {
      interleave(order, out);
    } else {
      size_t a = 0;
      while (a < order.size()) {
        const int g = d.env_sdf[d.inst_env[tiles[order[a]].inst]];
        size_t b = a;
        while (b < order.size() && d.env_sdf[d.inst_env[tiles[order[b]].inst]] == g) ++b;
        interleave(std::vector<int32_t>(order.begin() + a, order.begin() + b), out);
        a = b;
      }
    }
    order.swap(out);
  }
  return TACSL_OK;
}

template <class T>
hipError_t dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc((void**)p, count * sizeof(T));
}

template <class T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

}  // namespace

struct tacsl_plan_s {
  int device = 0;
  int32_t n_env = 0, n_inst = 0, n_tmpl = 0, n_sdf = 0;
  int64_t T = 0;
  int cu_count = 0;
  tacsl_tuning tun{};
  std::vector<int64_t> inst_off;
  // scene copies needed to rebuild the work list
  std::vector<int32_t> inst_env, inst_tmpl, env_sdf;
  std::vector<int32_t> sdf_dims;    // [n_sdf][3]
  std::vector<int64_t> grid_base;   // [n_sdf + 1] float4 offsets of the prepared grids
  std::vector<int64_t> tmpl_offset;
  const float* tmpl_xyz = nullptr;  // plan-owned copy of the templates
  int64_t tmpl_T = 0;
  float* d_tmpl = nullptr;  // plan-owned copy of the templates
  // device buffers
  float4* grids = nullptr;
  float* d_phi4 = nullptr;                 // node values in x-quad columns (depth image), built on demand
  tacsl::DepthGrid* d_dgrid = nullptr;     // [n_sdf]
  float4* d_slope = nullptr;               // per-grid block slope bounds (depth image), built with d_phi4
  int64_t slope_bytes = 0;
  // spatial pad order of the depth image (one unit per pad)
  uint32_t* d_dsp_hist = nullptr;
  uint32_t* d_dsp_cursor = nullptr;
  int32_t* d_dsp_bin = nullptr;
  int32_t* d_dsp_grp = nullptr;
  int64_t* d_dsp_units = nullptr;          // [n_inst + 1] = 0, 1, ..., n_inst
  int32_t* d_dsp_order = nullptr;          // [n_inst]
  int64_t phi4_bytes = 0;
  int64_t grids_bytes = 0;
  InstStatic* d_stat = nullptr;
  InstXf* d_xf = nullptr;
  Tile* d_tiles = nullptr;
  int32_t* d_order = nullptr;
  int64_t* d_inst_tile_begin = nullptr;
  float* d_partial = nullptr;
  double* d_bpartial = nullptr;
  int32_t* d_queue = nullptr;
  int32_t* d_env_inst_begin = nullptr;
  int32_t* d_env_inst = nullptr;
  float hc = 1.f;  // normal-law exponent (tacsl_plan_set_normal_law)
  // tactile camera (set by tacsl_plan_set_camera)
  bool has_cam = false;
  tacsl_camera cam{};
  // observation epilogue (set by tacsl_plan_set_observation)
  int32_t obs_n = 0;
  float obs_scale[3] = {1.f, 1.f, 1.f};
  float obs_clip = 0.f;
  int32_t* d_obs_bin = nullptr;      // [tmpl_T]
  float* d_obs_icnt = nullptr;       // [n_tmpl][obs_n]
  int32_t* d_obs_inst_tmpl = nullptr;  // [n_inst]
  float* d_obs_partial = nullptr;    // [n_tiles][obs_n][3]
  // spatial order (order 5)
  uint32_t* d_sp_hist = nullptr;
  uint32_t* d_sp_cursor = nullptr;
  int32_t* d_sp_bin = nullptr;
  int32_t* d_sp_grp_tile = nullptr;
  int64_t n_tiles = 0;
  // device bytes of everything but the prepared SDF pool (what is allocated now)
  int64_t workspace_bytes() const {
    const int64_t ni = n_inst, nt = n_tiles, ns = n_sdf;
    int64_t b = ni * (int64_t)(sizeof(InstStatic) + sizeof(InstXf)) + 3 * tmpl_T * (int64_t)sizeof(float) +
                nt * (int64_t)(sizeof(Tile) + sizeof(int32_t) + 6 * sizeof(float) + tacsl::kBwdAcc * sizeof(double)) +
                (ni + 1) * (int64_t)sizeof(int64_t) + (n_env + 1 + ni) * 4 + 4;
    if (obs_n > 0) b += tmpl_T * 4 + ns * obs_n * 4 + ni * 4 + nt * 3 * obs_n * 4;
    if (d_sp_hist) b += 2 * tacsl::kSpatialBins * ns * 4 + ni * 4 + (ns + 1) * 4;
    if (d_phi4) b += phi4_bytes + slope_bytes + ns * (int64_t)sizeof(tacsl::DepthGrid);
    if (d_dsp_hist) b += 2 * tacsl::kSpatialBins * ns * 4 + ni * 4 + (ns + 1) * 4 + (ni + 1) * 8 + ni * 4;
    return b;
  }
  int live_graphs = 0;
  // kernel timer (instrumentation)
  std::vector<hipEvent_t> ev_start, ev_stop;
  int32_t timer_n = 0;

  void free_timer() {
    for (hipEvent_t e : ev_start) (void)hipEventDestroy(e);
    for (hipEvent_t e : ev_stop) (void)hipEventDestroy(e);
    ev_start.clear();
    ev_stop.clear();
    timer_n = 0;
  }
  bool timing() const { return timer_n < (int32_t)ev_start.size(); }

  tacsl_scene_desc desc() const {
    tacsl_scene_desc d{};
    d.n_env = n_env;
    d.n_inst = n_inst;
    d.n_tmpl = n_tmpl;
    d.n_sdf = n_sdf;
    d.inst_env = inst_env.data();
    d.inst_tmpl = inst_tmpl.data();
    d.env_sdf = env_sdf.data();
    d.tmpl_offset = tmpl_offset.data();
    d.tmpl_xyz = tmpl_xyz;
    return d;
  }

  void free_worklist() {
    dfree(d_tiles);
    dfree(d_order);
    dfree(d_inst_tile_begin);
    dfree(d_partial);
    dfree(d_bpartial);
    dfree(d_obs_partial);
    dfree(d_sp_hist);
    dfree(d_sp_cursor);
    dfree(d_sp_bin);
    dfree(d_sp_grp_tile);
  }
  void free_observation() {
    dfree(d_obs_bin);
    dfree(d_obs_icnt);
    dfree(d_obs_inst_tmpl);
    dfree(d_obs_partial);
    obs_n = 0;
  }
  void free_all() {
    free_timer();
    free_worklist();
    dfree(d_tmpl);
    dfree(grids);
    dfree(d_stat);
    dfree(d_xf);
    dfree(d_queue);
    dfree(d_env_inst_begin);
    dfree(d_env_inst);
    dfree(d_phi4);
    dfree(d_dgrid);
    dfree(d_slope);
    dfree(d_dsp_hist);
    dfree(d_dsp_cursor);
    dfree(d_dsp_bin);
    dfree(d_dsp_grp);
    dfree(d_dsp_units);
    dfree(d_dsp_order);
    free_observation();
  }
};

struct tacsl_graph_s {
  std::vector<tacsl_plan> plans;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Device buffers of one work list; installed into a plan only when complete.
struct WorkBuffers {
  Tile* tiles = nullptr;
  int32_t* order = nullptr;
  int64_t* inst_tile_begin = nullptr;
  float* partial = nullptr;
  double* bpartial = nullptr;
  float* obs_partial = nullptr;
  uint32_t* sp_hist = nullptr;
  uint32_t* sp_cursor = nullptr;
  int32_t* sp_bin = nullptr;
  int32_t* sp_grp_tile = nullptr;
  void release() {
    dfree(tiles);
    dfree(order);
    dfree(inst_tile_begin);
    dfree(partial);
    dfree(bpartial);
    dfree(obs_partial);
    dfree(sp_hist);
    dfree(sp_cursor);
    dfree(sp_bin);
    dfree(sp_grp_tile);
  }
};

// Build and upload the work list of tuning t; the plan's previous work list
// stays in place (and usable) if anything fails.
int install_worklist(tacsl_plan p, const tacsl_tuning& t) {
  std::vector<Tile> tiles;
  std::vector<int32_t> order;
  std::vector<int64_t> itb;
  const tacsl_scene_desc d = p->desc();
  int rc = make_worklist(d, t, kXcdCount, tiles, order, itb);
  if (rc != TACSL_OK) return rc;
  const size_t n = tiles.size();
  WorkBuffers w;
  bool ok = dalloc(&w.tiles, n) == hipSuccess && dalloc(&w.order, n) == hipSuccess &&
            dalloc(&w.inst_tile_begin, itb.size()) == hipSuccess && dalloc(&w.partial, 6 * n) == hipSuccess &&
            dalloc(&w.bpartial, (size_t)tacsl::kBwdAcc * n) == hipSuccess &&
            (p->obs_n == 0 || dalloc(&w.obs_partial, (size_t)3 * p->obs_n * n) == hipSuccess);
  const size_t nb = (size_t)tacsl::kSpatialBins * std::max(p->n_sdf, 1);
  if (ok && t.order == 5)
    ok = dalloc(&w.sp_hist, nb) == hipSuccess && dalloc(&w.sp_cursor, nb) == hipSuccess &&
         dalloc(&w.sp_bin, (size_t)p->n_inst) == hipSuccess &&
         dalloc(&w.sp_grp_tile, (size_t)p->n_sdf + 1) == hipSuccess;
  if (!ok) {
    w.release();
    return TACSL_ERR_ALLOC;
  }
  ok = (t.order != 5 || hipMemset(w.sp_hist, 0, nb * sizeof(uint32_t)) == hipSuccess) &&
       (n == 0 || (hipMemcpy(w.tiles, tiles.data(), n * sizeof(Tile), hipMemcpyHostToDevice) == hipSuccess &&
                   hipMemcpy(w.order, order.data(), n * sizeof(int32_t), hipMemcpyHostToDevice) == hipSuccess)) &&
       hipMemcpy(w.inst_tile_begin, itb.data(), itb.size() * sizeof(int64_t), hipMemcpyHostToDevice) == hipSuccess;
  if (!ok) {
    w.release();
    return TACSL_ERR_HIP;
  }
  p->free_worklist();
  p->d_tiles = w.tiles;
  p->d_order = w.order;
  p->d_inst_tile_begin = w.inst_tile_begin;
  p->d_partial = w.partial;
  p->d_bpartial = w.bpartial;
  p->d_obs_partial = w.obs_partial;
  p->d_sp_hist = w.sp_hist;
  p->d_sp_cursor = w.sp_cursor;
  p->d_sp_bin = w.sp_bin;
  p->d_sp_grp_tile = w.sp_grp_tile;
  p->n_tiles = (int64_t)n;
  p->tun = t;
  return TACSL_OK;
}

// Buffers one forward call writes and reads back: the plan's own, or carved
// from the library's static device scratch (tacsl_force_field_noalloc).
struct CallBuffers {
  InstXf* xf;
  int32_t* queue;
  float* partial;
  int32_t* order;
  uint32_t* sp_hist;
  uint32_t* sp_cursor;
  int32_t* sp_bin;
  int32_t* sp_grp_tile;
};

CallBuffers plan_buffers(const tacsl_plan p) {
  return CallBuffers{p->d_xf, p->d_queue, p->d_partial, p->d_order,
                     p->d_sp_hist, p->d_sp_cursor, p->d_sp_bin, p->d_sp_grp_tile};
}

int64_t align256(int64_t b) { return (b + 255) / 256 * 256; }

// Bytes of static scratch a forward call of plan p needs.
int64_t scratch_bytes(const tacsl_plan p) {
  int64_t b = align256(4) + align256((int64_t)p->n_inst * (int64_t)sizeof(InstXf)) +
              align256(p->n_tiles * 6 * (int64_t)sizeof(float));
  if (p->tun.order == 5) {
    const int64_t nb = (int64_t)tacsl::kSpatialBins * std::max(p->n_sdf, 1);
    b += 2 * align256(nb * 4) + align256((int64_t)p->n_inst * 4) + align256(((int64_t)p->n_sdf + 1) * 4) +
         align256(p->n_tiles * 4);
  }
  return b;
}

// Carve the call buffers of plan p out of the scratch at `base` (order 5:
// the spatial histogram is cleared by a kernel on `stream` first).
int scratch_buffers(const tacsl_plan p, char* base, hipStream_t stream, CallBuffers* cb) {
  *cb = plan_buffers(p);
  char* q = base;
  auto take = [&](int64_t bytes) {
    char* r = q;
    q += align256(bytes);
    return r;
  };
  cb->queue = reinterpret_cast<int32_t*>(take(4));
  cb->xf = reinterpret_cast<InstXf*>(take((int64_t)p->n_inst * (int64_t)sizeof(InstXf)));
  cb->partial = reinterpret_cast<float*>(take(p->n_tiles * 6 * (int64_t)sizeof(float)));
  if (p->tun.order == 5) {
    const int64_t nb = (int64_t)tacsl::kSpatialBins * std::max(p->n_sdf, 1);
    cb->sp_hist = reinterpret_cast<uint32_t*>(take(nb * 4));
    cb->sp_cursor = reinterpret_cast<uint32_t*>(take(nb * 4));
    cb->sp_bin = reinterpret_cast<int32_t*>(take((int64_t)p->n_inst * 4));
    cb->sp_grp_tile = reinterpret_cast<int32_t*>(take(((int64_t)p->n_sdf + 1) * 4));
    cb->order = reinterpret_cast<int32_t*>(take(p->n_tiles * 4));
    if (tacsl::launch_zero_u32(cb->sp_hist, nb, stream) != hipSuccess) return TACSL_ERR_HIP;
  }
  return TACSL_OK;
}

// Spatial order (order 5): the prologue has binned the pads; rebuild the
// slot -> tile map for this call.
int enqueue_spatial(tacsl_plan p, hipStream_t stream, const CallBuffers* cb = nullptr) {
  if (p->tun.order != 5) return TACSL_OK;
  const CallBuffers b = cb ? *cb : plan_buffers(p);
  tacsl::SpatialArgs sa{};
  sa.n_inst = p->n_inst;
  sa.n_sdf = p->n_sdf;
  sa.n_tiles = (int32_t)p->n_tiles;
  sa.interleave = 1;
  sa.hist = b.sp_hist;
  sa.cursor = b.sp_cursor;
  sa.bin = b.sp_bin;
  sa.grp_tile_begin = b.sp_grp_tile;
  sa.inst_tile_begin = p->d_inst_tile_begin;
  sa.order = b.order;
  return tacsl::launch_spatial_order(sa, stream) == hipSuccess ? TACSL_OK : TACSL_ERR_HIP;
}

// Small launches (no more tiles than compute units) with orders 0-4 and a
// static or persistent schedule: the forward kernel computes each tile's pad
// record itself (its FP64 code raises the kernel to ~110 VGPRs, which only a
// launch of at most one workgroup per CU does not feel), so a call is one
// launch instead of two (plus the wrench reduction when pads span tiles).
bool fused_forward(const tacsl_plan p, const float* obs) {
  return obs == nullptr && p->tun.order != 5 && p->tun.schedule != 2 && p->n_tiles <= p->cu_count;
}

int enqueue_forward(tacsl_plan p, const tacsl_state* s, const tacsl_outputs* o, hipStream_t stream,
                    bool capturing, float* obs = nullptr, const CallBuffers* bufs = nullptr) {
  if (p->n_inst == 0) return TACSL_OK;
  const CallBuffers cb = bufs ? *bufs : plan_buffers(p);
  const bool fused = fused_forward(p, obs);
  tacsl::PrologueArgs pa{};
  pa.pad_pose = s->pad_pose;
  pa.obj_pose = s->obj_pose;
  pa.pad_twist = s->pad_twist;
  pa.obj_twist = s->obj_twist;
  pa.params = s->params;
  pa.obj_pose_delta = s->obj_pose_delta;
  pa.stat = p->d_stat;
  pa.xf = cb.xf;
  pa.n_inst = p->n_inst;
  pa.status = o->status;
  pa.queue = cb.queue;
  pa.hc = p->hc;
  if (p->tun.order == 5) {
    pa.sp_hist = cb.sp_hist;
    pa.sp_bin = cb.sp_bin;
    pa.sp_inst_tile_begin = p->d_inst_tile_begin;
  }
  if (!fused && tacsl::launch_prologue(pa, stream) != hipSuccess) return TACSL_ERR_HIP;
  int src = enqueue_spatial(p, stream, &cb);
  if (src != TACSL_OK) return src;
  const bool direct = p->n_tiles == p->n_inst;  // one tile per pad: tile id == pad id
  const bool fields = o->depth != nullptr;
  tacsl::FwdArgs fa{};
  fa.tiles = p->d_tiles;
  fa.order = cb.order;
  fa.n_tiles = (int32_t)p->n_tiles;
  fa.dynamic = p->tun.schedule == 2 ? 1 : 0;
  fa.queue = cb.queue;
  fa.stat = p->d_stat;
  fa.xf = cb.xf;
  fa.tmpl = p->tmpl_xyz;
  fa.tmpl_T = p->tmpl_T;
  fa.depth = o->depth;
  fa.normal = o->normal;
  fa.fn = o->fn;
  fa.ft = o->ft;
  fa.T = p->T;
  fa.partial = direct ? o->wrench : cb.partial;
  fa.mode = obs ? (fields ? 3 : 2) : 1;  // without the observation the fields are always written
  fa.nonlinear = p->hc != 1.f ? 1 : 0;
  fa.obs_bin = p->d_obs_bin;
  fa.obs_n = obs ? p->obs_n : 0;
  fa.obs_partial = p->d_obs_partial;
  fa.fused = fused ? 1 : 0;
  fa.fin = tacsl::FusedIn{s->pad_pose, s->obj_pose, s->pad_twist, s->obj_twist, s->params, s->obj_pose_delta,
                          o->status, p->hc};
  const int grid = p->tun.schedule == 0 ? (int)p->n_tiles : (int)std::min<int64_t>(p->tun.grid, p->n_tiles);
  bool timed = !capturing && p->timing();
  if (timed) {
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return TACSL_ERR_HIP;
    timed = cap == hipStreamCaptureStatusNone;
  }
  if (timed && hipEventRecord(p->ev_start[p->timer_n], stream) != hipSuccess) return TACSL_ERR_HIP;
  if (tacsl::launch_forward(fa, p->tun.block, grid, stream) != hipSuccess) return TACSL_ERR_HIP;
  if (timed) {
    if (hipEventRecord(p->ev_stop[p->timer_n], stream) != hipSuccess) return TACSL_ERR_HIP;
    p->timer_n++;
  }
  if (!direct) {
    tacsl::WrenchReduceArgs ra{p->d_inst_tile_begin, cb.partial, o->wrench, p->n_inst};
    if (tacsl::launch_wrench_reduce(ra, stream) != hipSuccess) return TACSL_ERR_HIP;
  }
  if (obs) {
    tacsl::ObsReduceArgs oa{};
    oa.inst_tile_begin = p->d_inst_tile_begin;
    oa.partial = p->d_obs_partial;
    oa.inst_tmpl = p->d_obs_inst_tmpl;
    oa.icnt = p->d_obs_icnt;
    for (int c = 0; c < 3; ++c) oa.scale[c] = p->obs_scale[c];
    oa.clip = p->obs_clip;
    oa.obs_n = p->obs_n;
    oa.n_inst = p->n_inst;
    oa.obs = obs;
    if (tacsl::launch_obs_reduce(oa, stream) != hipSuccess) return TACSL_ERR_HIP;
  }
  return TACSL_OK;
}

int check_state(const tacsl_plan p, const tacsl_state* s) {
  if (!s) return TACSL_ERR_NULL_ARG;
  if (p->n_inst > 0 && (!s->pad_pose || !s->obj_pose || !s->pad_twist || !s->obj_twist || !s->params))
    return TACSL_ERR_NULL_ARG;
  return TACSL_OK;
}

int check_outputs(const tacsl_plan p, const tacsl_outputs* o) {
  if (!o) return TACSL_ERR_NULL_ARG;
  if (p->n_inst > 0 && (!o->wrench || (p->T > 0 && (!o->depth || !o->normal || !o->fn || !o->ft))))
    return TACSL_ERR_NULL_ARG;
  return TACSL_OK;
}

}  // namespace

extern "C" {

int tacsl_abi_version(void) { return TACSL_ABI_VERSION; }

const char* tacsl_status_string(int status) {
  switch (status) {
    case TACSL_OK: return "TACSL_OK";
    case TACSL_ERR_NULL_ARG: return "TACSL_ERR_NULL_ARG: a required pointer is NULL";
    case TACSL_ERR_SHAPE: return "TACSL_ERR_SHAPE: inconsistent counts or offsets";
    case TACSL_ERR_RANGE: return "TACSL_ERR_RANGE: id or value out of range";
    case TACSL_ERR_HIP: return "TACSL_ERR_HIP: HIP runtime call failed";
    case TACSL_ERR_ALLOC: return "TACSL_ERR_ALLOC: allocation failed";
    case TACSL_ERR_UNSUPPORTED: return "TACSL_ERR_UNSUPPORTED: beyond this build's limits";
    case TACSL_ERR_STATE: return "TACSL_ERR_STATE: call not valid for this object";
    default: return "TACSL_ERR_UNKNOWN";
  }
}

int tacsl_validate_scene(const tacsl_scene_desc* desc) { return validate(desc); }

int tacsl_build_worklist(const tacsl_scene_desc* desc, const tacsl_tuning* tuning, int32_t xcd_count,
                         int64_t max_tiles, int64_t* n_tiles, int32_t* tile_inst, int32_t* tile_k0,
                         int32_t* tile_count, int32_t* exec_order) {
  int rc = validate(desc);
  if (rc != TACSL_OK) return rc;
  if (!n_tiles) return TACSL_ERR_NULL_ARG;
  if (xcd_count < 1) return TACSL_ERR_RANGE;
  tacsl_tuning t;
  rc = resolve_tuning(tuning, 1, &t);
  if (rc != TACSL_OK) return rc;
  std::vector<Tile> tiles;
  std::vector<int32_t> order;
  std::vector<int64_t> itb;
  rc = make_worklist(*desc, t, xcd_count, tiles, order, itb);
  if (rc != TACSL_OK) return rc;
  *n_tiles = (int64_t)tiles.size();
  if (!tile_inst && !tile_k0 && !tile_count && !exec_order) return TACSL_OK;
  if (!tile_inst || !tile_k0 || !tile_count || !exec_order) return TACSL_ERR_NULL_ARG;
  if ((int64_t)tiles.size() > max_tiles) return TACSL_ERR_SHAPE;
  for (size_t k = 0; k < tiles.size(); ++k) {
    tile_inst[k] = tiles[k].inst;
    tile_k0[k] = tiles[k].k0;
    tile_count[k] = tiles[k].count;
    exec_order[k] = order[k];
  }
  return TACSL_OK;
}

int tacsl_plan_create(const tacsl_scene_desc* desc, const tacsl_tuning* tuning, tacsl_plan* out) {
  const Range range("tacsl_plan_create");
  if (!out) return TACSL_ERR_NULL_ARG;
  *out = nullptr;
  int rc = validate(desc);
  if (rc != TACSL_OK) return rc;
  tacsl_plan p = new (std::nothrow) tacsl_plan_s();
  if (!p) return TACSL_ERR_ALLOC;
  auto fail = [&](int code) {
    p->free_all();
    delete p;
    return code;
  };
  if (hipGetDevice(&p->device) != hipSuccess) return fail(TACSL_ERR_HIP);
  if (hipDeviceGetAttribute(&p->cu_count, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess)
    return fail(TACSL_ERR_HIP);
  tacsl_tuning t;
  rc = resolve_tuning(tuning, p->cu_count, &t);
  if (rc != TACSL_OK) return fail(rc);
  const tacsl_scene_desc& d = *desc;
  p->n_env = d.n_env;
  p->n_inst = d.n_inst;
  p->n_tmpl = d.n_tmpl;
  p->n_sdf = d.n_sdf;
  p->inst_env.assign(d.inst_env, d.inst_env + d.n_inst);
  p->inst_tmpl.assign(d.inst_tmpl, d.inst_tmpl + d.n_inst);
  p->env_sdf.assign(d.env_sdf, d.env_sdf + d.n_env);
  p->tmpl_offset.assign(d.tmpl_offset, d.tmpl_offset + (d.n_tmpl > 0 ? d.n_tmpl + 1 : 0));
  p->tmpl_T = d.n_tmpl > 0 ? d.tmpl_offset[d.n_tmpl] : 0;
  // plan-owned copy of the templates (taxels are visited in the caller's
  // order, so a compact numbering -- e.g. 8 x 8 blocks -- gives compact waves)
  {
    const int64_t TT = p->tmpl_T;
    if (dalloc(&p->d_tmpl, (size_t)(3 * TT)) != hipSuccess) return fail(TACSL_ERR_ALLOC);
    if (TT > 0 && hipMemcpy(p->d_tmpl, d.tmpl_xyz, (size_t)(3 * TT) * sizeof(float), hipMemcpyDeviceToDevice) !=
                      hipSuccess)
      return fail(TACSL_ERR_HIP);
    p->tmpl_xyz = p->d_tmpl;
  }
  p->inst_off.assign((size_t)d.n_inst + 1, 0);
  for (int i = 0; i < d.n_inst; ++i) p->inst_off[i + 1] = p->inst_off[i] + tmpl_count(d, i);
  p->T = p->inst_off[d.n_inst];

  // prepared SDF pool: per grid, (phi, G) float4 records in 2 x 2 columns and
  // the clear-block mask after them
  std::vector<int64_t> gbase((size_t)d.n_sdf + 1, 0);
  for (int g = 0; g < d.n_sdf; ++g)
    gbase[g + 1] = gbase[g] + tacsl::prepared_grid_bytes(d.sdf_dims[3 * g], d.sdf_dims[3 * g + 1],
                                                         d.sdf_dims[3 * g + 2]) / (int64_t)sizeof(float4);
  p->grids_bytes = gbase[d.n_sdf] * (int64_t)sizeof(float4);
  p->grid_base = gbase;
  p->sdf_dims.assign(d.sdf_dims, d.sdf_dims + 3 * d.n_sdf);
  if (dalloc(&p->grids, (size_t)gbase[d.n_sdf]) != hipSuccess) return fail(TACSL_ERR_ALLOC);
  uint32_t* d_bad = nullptr;
  if (dalloc(&d_bad, 1) != hipSuccess) return fail(TACSL_ERR_ALLOC);
  if (hipMemset(d_bad, 0, sizeof(uint32_t)) != hipSuccess) {
    dfree(d_bad);
    return fail(TACSL_ERR_HIP);
  }
  for (int g = 0; g < d.n_sdf; ++g) {
    const int nx = d.sdf_dims[3 * g], ny = d.sdf_dims[3 * g + 1], nz = d.sdf_dims[3 * g + 2];
    uint32_t* mask = reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(p->grids + gbase[g]) +
                                                 tacsl::grid_record_bytes(nx, ny, nz));
    if (tacsl::launch_prepare_grid(d.sdf_data + d.sdf_offset[g], p->grids + gbase[g], nx, ny, nz, d.sdf_spacing[g],
                                   d_bad, nullptr) != hipSuccess ||
        tacsl::launch_clear_mask(d.sdf_data + d.sdf_offset[g], mask, nx, ny, nz, nullptr) != hipSuccess) {
      dfree(d_bad);
      return fail(TACSL_ERR_HIP);
    }
  }
  uint32_t bad = 0;
  hipError_t e = hipMemcpy(&bad, d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost);
  dfree(d_bad);
  if (e != hipSuccess) return fail(TACSL_ERR_HIP);
  if (bad) return fail(TACSL_ERR_RANGE);
  // static per-pad records
  std::vector<InstStatic> st((size_t)d.n_inst);
  for (int i = 0; i < d.n_inst; ++i) {
    const int g = d.env_sdf[d.inst_env[i]];
    InstStatic& s = st[i];
    s.grid = p->grids + gbase[g];
    s.tmpl_off = d.tmpl_offset[d.inst_tmpl[i]];
    s.out_off = p->inst_off[i];
    s.nx = d.sdf_dims[3 * g];
    s.ny = d.sdf_dims[3 * g + 1];
    s.nz = d.sdf_dims[3 * g + 2];
    s.env = d.inst_env[i];
    s.count = (int32_t)tmpl_count(d, i);
    s.grid_bytes = (uint32_t)((gbase[g + 1] - gbase[g]) * (int64_t)sizeof(float4));
    s.stride_y = 64u * (uint32_t)s.nz;
    s.stride_q = s.stride_y * (uint32_t)((s.ny + 1) / 2);
    s.ox = d.sdf_origin[3 * g];
    s.oy = d.sdf_origin[3 * g + 1];
    s.oz = d.sdf_origin[3 * g + 2];
    s.h = d.sdf_spacing[g];
    s.gid = g;
    const tacsl::MaskDims md = tacsl::mask_dims(s.nx, s.ny, s.nz);
    s.mask_off = (uint32_t)tacsl::grid_record_bytes(s.nx, s.ny, s.nz);
    s.mask_sx = (uint32_t)(4 * md.wy * md.wz);
    s.mask_sy = (uint32_t)(4 * md.wz);
  }
  // environments -> pads (ascending)
  std::vector<int32_t> eib((size_t)d.n_env + 1, 0), ei((size_t)d.n_inst);
  for (int i = 0; i < d.n_inst; ++i) eib[d.inst_env[i] + 1]++;
  for (int e2 = 0; e2 < d.n_env; ++e2) eib[e2 + 1] += eib[e2];
  {
    std::vector<int32_t> fill(eib.begin(), eib.end() - 1);
    for (int i = 0; i < d.n_inst; ++i) ei[fill[d.inst_env[i]]++] = i;
  }
  if (dalloc(&p->d_stat, st.size()) != hipSuccess || dalloc(&p->d_xf, (size_t)d.n_inst) != hipSuccess ||
      dalloc(&p->d_queue, 1) != hipSuccess || dalloc(&p->d_env_inst_begin, eib.size()) != hipSuccess ||
      dalloc(&p->d_env_inst, ei.size()) != hipSuccess)
    return fail(TACSL_ERR_ALLOC);
  if ((!st.empty() && hipMemcpy(p->d_stat, st.data(), st.size() * sizeof(InstStatic), hipMemcpyHostToDevice) !=
                          hipSuccess) ||
      hipMemcpy(p->d_env_inst_begin, eib.data(), eib.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
          hipSuccess ||
      (!ei.empty() && hipMemcpy(p->d_env_inst, ei.data(), ei.size() * sizeof(int32_t), hipMemcpyHostToDevice) !=
                          hipSuccess) ||
      hipMemset(p->d_queue, 0, sizeof(int32_t)) != hipSuccess)
    return fail(TACSL_ERR_HIP);
  rc = install_worklist(p, t);
  if (rc != TACSL_OK) return fail(rc);
  if (hipDeviceSynchronize() != hipSuccess) return fail(TACSL_ERR_HIP);
  *out = p;
  return TACSL_OK;
}

int tacsl_plan_set_tuning(tacsl_plan plan, const tacsl_tuning* tuning) {
  const Range range("tacsl_plan_set_tuning");
  if (!plan) return TACSL_ERR_NULL_ARG;
  if (plan->live_graphs > 0) return TACSL_ERR_STATE;
  tacsl_tuning t;
  int rc = resolve_tuning(tuning, plan->cu_count, &t);
  if (rc != TACSL_OK) return rc;
  if (hipDeviceSynchronize() != hipSuccess) return TACSL_ERR_HIP;
  return install_worklist(plan, t);
}

int tacsl_plan_get_info(tacsl_plan plan, tacsl_plan_info* info) {
  if (!plan || !info) return TACSL_ERR_NULL_ARG;
  info->n_taxels = plan->T;
  info->n_tiles = plan->n_tiles;
  info->n_env = plan->n_env;
  info->n_inst = plan->n_inst;
  info->cu_count = plan->cu_count;
  info->xcd_count = kXcdCount;
  info->prepared_bytes = plan->grids_bytes;
  info->workspace_bytes = plan->workspace_bytes();
  info->tuning = plan->tun;
  return TACSL_OK;
}

int tacsl_plan_offsets(tacsl_plan plan, int64_t* host_inst_offset) {
  if (!plan || !host_inst_offset) return TACSL_ERR_NULL_ARG;
  std::memcpy(host_inst_offset, plan->inst_off.data(), plan->inst_off.size() * sizeof(int64_t));
  return TACSL_OK;
}

int tacsl_force_field(tacsl_plan plan, const tacsl_state* state, const tacsl_outputs* out, hipStream_t stream) {
  const Range range("tacsl_force_field");
  if (!plan) return TACSL_ERR_NULL_ARG;
  int rc = check_state(plan, state);
  if (rc != TACSL_OK) return rc;
  rc = check_outputs(plan, out);
  if (rc != TACSL_OK) return rc;
  return enqueue_forward(plan, state, out, stream, false);
}

int tacsl_force_field_noalloc(tacsl_plan plan, const tacsl_state* state, const tacsl_outputs* out,
                              hipStream_t stream) {
  const Range range("tacsl_force_field_noalloc");
  if (!plan) return TACSL_ERR_NULL_ARG;
  int rc = check_state(plan, state);
  if (rc != TACSL_OK) return rc;
  rc = check_outputs(plan, out);
  if (rc != TACSL_OK) return rc;
  if (plan->n_inst == 0) return TACSL_OK;
  if (scratch_bytes(plan) > tacsl::kScratchBytes) return TACSL_ERR_UNSUPPORTED;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return TACSL_ERR_HIP;
  if (dev != plan->device) return TACSL_ERR_STATE;
  void* base = nullptr;
  const hipError_t e = tacsl::scratch_address(dev, &base);
  if (e == hipErrorInvalidDevice) return TACSL_ERR_UNSUPPORTED;
  if (e != hipSuccess || !base) return TACSL_ERR_HIP;
  CallBuffers cb{};
  rc = scratch_buffers(plan, static_cast<char*>(base), stream, &cb);
  if (rc != TACSL_OK) return rc;
  return enqueue_forward(plan, state, out, stream, false, nullptr, &cb);
}

int tacsl_plan_set_observation(tacsl_plan plan, int32_t n_bins, const int32_t* tmpl_bin, const float* scale,
                               float clip) {
  const Range range("tacsl_plan_set_observation");
  if (!plan) return TACSL_ERR_NULL_ARG;
  if (plan->live_graphs > 0) return TACSL_ERR_STATE;
  if (n_bins == 0) {
    if (hipDeviceSynchronize() != hipSuccess) return TACSL_ERR_HIP;
    plan->free_observation();
    return TACSL_OK;
  }
  if (n_bins < 0 || n_bins > TACSL_MAX_OBS_BINS) return TACSL_ERR_RANGE;
  if (!scale || (plan->tmpl_T > 0 && !tmpl_bin)) return TACSL_ERR_NULL_ARG;
  for (int c = 0; c < 3; ++c)
    if (!(scale[c] > 0.f) || !std::isfinite(scale[c])) return TACSL_ERR_RANGE;
  if (!std::isfinite(clip)) return TACSL_ERR_RANGE;
  const int64_t TT = plan->tmpl_T;
  std::vector<float> icnt((size_t)plan->n_tmpl * n_bins, 0.f);
  for (int p = 0; p < plan->n_tmpl; ++p) {
    for (int64_t k = plan->tmpl_offset[p]; k < plan->tmpl_offset[p + 1]; ++k) {
      const int32_t b = tmpl_bin[k];
      if (b < -1 || b >= n_bins) return TACSL_ERR_RANGE;
      if (b >= 0) icnt[(size_t)p * n_bins + b] += 1.f;
    }
  }
  for (float& v : icnt) v = v > 0.f ? 1.f / v : 0.f;
  if (hipDeviceSynchronize() != hipSuccess) return TACSL_ERR_HIP;
  plan->free_observation();
  if (dalloc(&plan->d_obs_bin, (size_t)TT) != hipSuccess || dalloc(&plan->d_obs_icnt, icnt.size()) != hipSuccess ||
      dalloc(&plan->d_obs_inst_tmpl, (size_t)plan->n_inst) != hipSuccess ||
      dalloc(&plan->d_obs_partial, (size_t)3 * n_bins * plan->n_tiles) != hipSuccess) {
    plan->free_observation();
    return TACSL_ERR_ALLOC;
  }
  if ((TT > 0 && hipMemcpy(plan->d_obs_bin, tmpl_bin, (size_t)TT * sizeof(int32_t), hipMemcpyHostToDevice) !=
                     hipSuccess) ||
      (!icnt.empty() && hipMemcpy(plan->d_obs_icnt, icnt.data(), icnt.size() * sizeof(float),
                                  hipMemcpyHostToDevice) != hipSuccess) ||
      (plan->n_inst > 0 && hipMemcpy(plan->d_obs_inst_tmpl, plan->inst_tmpl.data(),
                                     (size_t)plan->n_inst * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess)) {
    plan->free_observation();
    return TACSL_ERR_HIP;
  }
  plan->obs_n = n_bins;
  for (int c = 0; c < 3; ++c) plan->obs_scale[c] = scale[c];
  plan->obs_clip = clip;
  return TACSL_OK;
}

int tacsl_force_field_observe(tacsl_plan plan, const tacsl_state* state, const tacsl_outputs* out, float* obs,
                              hipStream_t stream) {
  const Range range("tacsl_force_field_observe");
  if (!plan) return TACSL_ERR_NULL_ARG;
  if (plan->obs_n == 0) return TACSL_ERR_STATE;
  int rc = check_state(plan, state);
  if (rc != TACSL_OK) return rc;
  if (!out) return TACSL_ERR_NULL_ARG;
  const int given = (out->depth != nullptr) + (out->normal != nullptr) + (out->fn != nullptr) + (out->ft != nullptr);
  if (given != 0 && given != 4) return TACSL_ERR_NULL_ARG;
  if (plan->n_inst > 0 && (!out->wrench || !obs)) return TACSL_ERR_NULL_ARG;
  if (given == 4) {
    rc = check_outputs(plan, out);
    if (rc != TACSL_OK) return rc;
  }
  return enqueue_forward(plan, state, out, stream, false, obs);
}

int tacsl_plan_set_normal_law(tacsl_plan plan, float exponent) {
  if (!plan) return TACSL_ERR_NULL_ARG;
  if (!(exponent >= 1.f && exponent <= 4.f)) return TACSL_ERR_RANGE;
  if (plan->live_graphs > 0) return TACSL_ERR_STATE;
  plan->hc = exponent;
  return TACSL_OK;
}

int tacsl_plan_set_camera(tacsl_plan plan, const tacsl_camera* cam) {
  const Range range("tacsl_plan_set_camera");
  if (!plan) return TACSL_ERR_NULL_ARG;
  if (!cam) {
    plan->has_cam = false;
    return TACSL_OK;
  }
  const tacsl_camera& c = *cam;
  if (c.rows < 1 || c.rows > 4096 || c.cols < 1 || c.cols > 4096 || (c.ortho != 0 && c.ortho != 1))
    return TACSL_ERR_RANGE;
  const float f[] = {c.x0, c.y0, c.dx, c.dy, c.cam_dist, c.gel};
  for (float v : f)
    if (!std::isfinite(v)) return TACSL_ERR_RANGE;
  if (!(c.dx > 0.f) || !(c.dy > 0.f) || !(c.gel > 0.f) || !(c.cam_dist >= c.gel)) return TACSL_ERR_RANGE;
  if (!plan->d_phi4 && plan->n_sdf > 0) {
    // node values in x-quad columns and block slope bounds for the ray march (built once)
    std::vector<tacsl::DepthGrid> dg((size_t)plan->n_sdf);
    std::vector<int64_t> base((size_t)plan->n_sdf + 1, 0), sbase((size_t)plan->n_sdf + 1, 0);
    int64_t smax = 0;
    for (int g = 0; g < plan->n_sdf; ++g) {
      const int64_t nx = plan->sdf_dims[3 * g], ny = plan->sdf_dims[3 * g + 1], nz = plan->sdf_dims[3 * g + 2];
      base[g + 1] = base[g] + tacsl::phi_quad_bytes(nx, ny, nz) / (int64_t)sizeof(float);
      const int64_t nb = tacsl::slope_blocks(nx) * tacsl::slope_blocks(ny) * tacsl::slope_blocks(nz);
      sbase[g + 1] = sbase[g] + nb;
      smax = std::max(smax, nb);
    }
    float* d_phi4 = nullptr;
    float4 *d_slope = nullptr, *d_raw = nullptr;
    tacsl::DepthGrid* d_dg = nullptr;
    auto release = [&]() {
      dfree(d_phi4);
      dfree(d_slope);
      dfree(d_raw);
      dfree(d_dg);
    };
    if (hipDeviceSynchronize() != hipSuccess) return TACSL_ERR_HIP;
    if (dalloc(&d_phi4, (size_t)base[plan->n_sdf]) != hipSuccess || dalloc(&d_dg, dg.size()) != hipSuccess ||
        dalloc(&d_slope, (size_t)sbase[plan->n_sdf]) != hipSuccess || dalloc(&d_raw, (size_t)smax) != hipSuccess) {
      release();
      return TACSL_ERR_ALLOC;
    }
    bool ok = hipMemset(d_phi4, 0, (size_t)base[plan->n_sdf] * sizeof(float)) == hipSuccess;
    for (int g = 0; ok && g < plan->n_sdf; ++g) {
      const int nx = plan->sdf_dims[3 * g], ny = plan->sdf_dims[3 * g + 1], nz = plan->sdf_dims[3 * g + 2];
      dg[g].phi = d_phi4 + base[g];
      dg[g].slope = d_slope + sbase[g];
      dg[g].bytes = (uint32_t)((base[g + 1] - base[g]) * (int64_t)sizeof(float));
      dg[g].stride_y = 16u * (uint32_t)nz;
      dg[g].stride_q = dg[g].stride_y * (uint32_t)ny;
      dg[g].sby = (int32_t)tacsl::slope_blocks(ny);
      dg[g].sbz = (int32_t)tacsl::slope_blocks(nz);
      dg[g].pad_ = 0;
      ok = tacsl::launch_phi_quad(plan->grids + plan->grid_base[g], nx, ny, nz, d_phi4 + base[g], nullptr) ==
               hipSuccess &&
           tacsl::launch_block_slopes(d_phi4 + base[g], nx, ny, nz, d_raw, d_slope + sbase[g], nullptr) == hipSuccess;
    }
    ok = ok && hipMemcpy(d_dg, dg.data(), dg.size() * sizeof(tacsl::DepthGrid), hipMemcpyHostToDevice) == hipSuccess &&
         hipDeviceSynchronize() == hipSuccess;
    dfree(d_raw);
    if (!ok) {
      release();
      return TACSL_ERR_HIP;
    }
    plan->d_phi4 = d_phi4;
    plan->d_dgrid = d_dg;
    plan->d_slope = d_slope;
    plan->phi4_bytes = base[plan->n_sdf] * (int64_t)sizeof(float);
    plan->slope_bytes = sbase[plan->n_sdf] * (int64_t)sizeof(float4);
  }
  if (!plan->d_dsp_order && plan->n_inst > 0) {
    const size_t nb = (size_t)tacsl::kSpatialBins * plan->n_sdf, ni = (size_t)plan->n_inst;
    std::vector<int64_t> units(ni + 1);
    std::iota(units.begin(), units.end(), int64_t(0));
    std::vector<int32_t> ident(ni);
    std::iota(ident.begin(), ident.end(), 0);
    bool ok = dalloc(&plan->d_dsp_hist, nb) == hipSuccess && dalloc(&plan->d_dsp_cursor, nb) == hipSuccess &&
              dalloc(&plan->d_dsp_bin, ni) == hipSuccess && dalloc(&plan->d_dsp_grp, (size_t)plan->n_sdf + 1) == hipSuccess &&
              dalloc(&plan->d_dsp_units, ni + 1) == hipSuccess && dalloc(&plan->d_dsp_order, ni) == hipSuccess;
    ok = ok && hipMemset(plan->d_dsp_hist, 0, nb * sizeof(uint32_t)) == hipSuccess &&
         hipMemcpy(plan->d_dsp_units, units.data(), units.size() * sizeof(int64_t), hipMemcpyHostToDevice) ==
             hipSuccess &&
         hipMemcpy(plan->d_dsp_order, ident.data(), ident.size() * sizeof(int32_t), hipMemcpyHostToDevice) ==
             hipSuccess;
    if (!ok) {
      dfree(plan->d_dsp_hist);
      dfree(plan->d_dsp_cursor);
      dfree(plan->d_dsp_bin);
      dfree(plan->d_dsp_grp);
      dfree(plan->d_dsp_units);
      dfree(plan->d_dsp_order);
      return TACSL_ERR_ALLOC;
    }
  }
  plan->cam = c;
  plan->has_cam = true;
  return TACSL_OK;
}

int tacsl_depth_image(tacsl_plan plan, const tacsl_state* state, float* image, uint32_t* status,
                      hipStream_t stream) {
  const Range range("tacsl_depth_image");
  if (!plan) return TACSL_ERR_NULL_ARG;
  if (!plan->has_cam) return TACSL_ERR_STATE;
  int rc = check_state(plan, state);
  if (rc != TACSL_OK) return rc;
  if (plan->n_inst == 0) return TACSL_OK;
  if (!image) return TACSL_ERR_NULL_ARG;
  tacsl::PrologueArgs pa{};
  pa.pad_pose = state->pad_pose;
  pa.obj_pose = state->obj_pose;
  pa.pad_twist = state->pad_twist;
  pa.obj_twist = state->obj_twist;
  pa.params = state->params;
  pa.obj_pose_delta = state->obj_pose_delta;
  pa.stat = plan->d_stat;
  pa.xf = plan->d_xf;
  pa.n_inst = plan->n_inst;
  pa.status = status;
  pa.queue = plan->d_queue;
  pa.hc = plan->hc;
  pa.sp_hist = plan->d_dsp_hist;
  pa.sp_bin = plan->d_dsp_bin;
  pa.sp_inst_tile_begin = plan->d_dsp_units;
  if (tacsl::launch_prologue(pa, stream) != hipSuccess) return TACSL_ERR_HIP;
  // pads in spatial order, object by object, each object's run cut into
  // one share per XCD (pad slot s is drawn by XCD s % 8)
  tacsl::SpatialArgs sa{};
  sa.n_inst = plan->n_inst;
  sa.n_sdf = plan->n_sdf;
  sa.n_tiles = plan->n_inst;
  sa.interleave = 1;
  sa.hist = plan->d_dsp_hist;
  sa.cursor = plan->d_dsp_cursor;
  sa.bin = plan->d_dsp_bin;
  sa.grp_tile_begin = plan->d_dsp_grp;
  sa.inst_tile_begin = plan->d_dsp_units;
  sa.order = plan->d_dsp_order;
  if (tacsl::launch_spatial_order(sa, stream) != hipSuccess) return TACSL_ERR_HIP;
  const tacsl_camera& c = plan->cam;
  tacsl::DepthArgs da{};
  da.stat = plan->d_stat;
  da.xf = plan->d_xf;
  da.grids = plan->d_dgrid;
  da.pad_order = plan->d_dsp_order;
  da.n_inst = plan->n_inst;
  da.rows = c.rows;
  da.cols = c.cols;
  da.ortho = c.ortho;
  da.x0 = c.x0;
  da.y0 = c.y0;
  da.dx = c.dx;
  da.dy = c.dy;
  da.cam_dist = c.cam_dist;
  da.gel = c.gel;
  da.blocks_x = (c.cols + 7) / 8;
  da.blocks_per_pad = da.blocks_x * ((c.rows + 7) / 8);
  da.image = image;
  da.status = status;
  return tacsl::launch_depth_image(da, stream) == hipSuccess ? TACSL_OK : TACSL_ERR_HIP;
}

int tacsl_force_field_backward(tacsl_plan plan, const tacsl_state* state, const tacsl_grads* g,
                               hipStream_t stream) {
  const Range range("tacsl_force_field_backward");
  if (!plan) return TACSL_ERR_NULL_ARG;
  int rc = check_state(plan, state);
  if (rc != TACSL_OK) return rc;
  if (!g) return TACSL_ERR_NULL_ARG;
  if (plan->n_env > 0 && (!g->g_obj_pose || !g->g_obj_twist || !g->g_params)) return TACSL_ERR_NULL_ARG;
  if (plan->T > 0 && (!g->w_fn || !g->w_ft)) return TACSL_ERR_NULL_ARG;
  if (plan->n_env == 0) return TACSL_OK;
  if (plan->n_inst > 0) {
    tacsl::PrologueArgs pa{};
    pa.pad_pose = state->pad_pose;
    pa.obj_pose = state->obj_pose;
    pa.pad_twist = state->pad_twist;
    pa.obj_twist = state->obj_twist;
    pa.params = state->params;
    pa.obj_pose_delta = state->obj_pose_delta;
    pa.stat = plan->d_stat;
    pa.xf = plan->d_xf;
    pa.n_inst = plan->n_inst;
    pa.status = g->status;
    pa.queue = plan->d_queue;
    pa.hc = plan->hc;
    if (plan->tun.order == 5) {
      pa.sp_hist = plan->d_sp_hist;
      pa.sp_bin = plan->d_sp_bin;
      pa.sp_inst_tile_begin = plan->d_inst_tile_begin;
    }
    if (tacsl::launch_prologue(pa, stream) != hipSuccess) return TACSL_ERR_HIP;
    rc = enqueue_spatial(plan, stream);
    if (rc != TACSL_OK) return rc;
    tacsl::BwdArgs ba{};
    ba.tiles = plan->d_tiles;
    ba.order = plan->d_order;
    ba.n_tiles = (int32_t)plan->n_tiles;
    ba.dynamic = plan->tun.schedule == 2 ? 1 : 0;
    ba.queue = plan->d_queue;
    ba.stat = plan->d_stat;
    ba.xf = plan->d_xf;
    ba.tmpl = plan->tmpl_xyz;
    ba.tmpl_T = plan->tmpl_T;
    ba.w_fn = g->w_fn;
    ba.w_ft = g->w_ft;
    ba.T = plan->T;
    ba.partial = plan->d_bpartial;
    ba.nonlinear = plan->hc != 1.f ? 1 : 0;
    const int grid =
        plan->tun.schedule == 0 ? (int)plan->n_tiles : (int)std::min<int64_t>(plan->tun.grid, plan->n_tiles);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(stream, &cap) != hipSuccess) return TACSL_ERR_HIP;
    const bool timed = cap == hipStreamCaptureStatusNone && plan->timing();
    if (timed && hipEventRecord(plan->ev_start[plan->timer_n], stream) != hipSuccess) return TACSL_ERR_HIP;
    if (tacsl::launch_backward(ba, plan->tun.block, grid, stream) != hipSuccess) return TACSL_ERR_HIP;
    if (timed) {
      if (hipEventRecord(plan->ev_stop[plan->timer_n], stream) != hipSuccess) return TACSL_ERR_HIP;
      plan->timer_n++;
    }
  }
  tacsl::GradReduceArgs ga{};
  ga.env_inst_begin = plan->d_env_inst_begin;
  ga.env_inst = plan->d_env_inst;
  ga.inst_tile_begin = plan->d_inst_tile_begin;
  ga.partial = plan->d_bpartial;
  ga.stat = plan->d_stat;
  ga.pad_pose = state->pad_pose;
  ga.obj_pose = state->obj_pose;
  ga.obj_twist = state->obj_twist;
  ga.obj_pose_delta = state->obj_pose_delta;
  ga.g_obj_pose = g->g_obj_pose;
  ga.g_obj_twist = g->g_obj_twist;
  ga.g_params = g->g_params;
  ga.n_env = plan->n_env;
  if (tacsl::launch_grad_reduce(ga, stream) != hipSuccess) return TACSL_ERR_HIP;
  return TACSL_OK;
}

int tacsl_pose_step(int32_t n_env, const float* pose0, const float* twist, double t, float* pose,
                    hipStream_t stream) {
  const Range range("tacsl_pose_step");
  if (n_env < 0) return TACSL_ERR_SHAPE;
  if (n_env == 0) return TACSL_OK;
  if (!pose0 || !twist || !pose) return TACSL_ERR_NULL_ARG;
  if (!std::isfinite(t)) return TACSL_ERR_RANGE;
  return tacsl::launch_pose_step(pose0, twist, t, n_env, pose, stream) == hipSuccess ? TACSL_OK : TACSL_ERR_HIP;
}

int tacsl_graph_create(int32_t n_plans, const tacsl_plan* plans, int32_t n_steps, const tacsl_state* states,
                       const tacsl_outputs* outs, tacsl_graph* out) {
  return tacsl_graph_create_path(n_plans, plans, n_steps, nullptr, states, outs, out);
}

int tacsl_graph_create_path(int32_t n_plans, const tacsl_plan* plans, int32_t n_steps, const tacsl_pose_path* paths,
                            const tacsl_state* states, const tacsl_outputs* outs, tacsl_graph* out) {
  const Range range("tacsl_graph_create_path");
  if (!out) return TACSL_ERR_NULL_ARG;
  *out = nullptr;
  if (!plans || !states || !outs) return TACSL_ERR_NULL_ARG;
  if (paths)
    for (int p = 0; p < n_plans; ++p)
      if (paths[p].poses && (!paths[p].pose0 || !paths[p].twist || !std::isfinite(paths[p].dt)))
        return paths[p].pose0 && paths[p].twist ? TACSL_ERR_RANGE : TACSL_ERR_NULL_ARG;
  if (n_plans < 1 || n_steps < 1) return TACSL_ERR_SHAPE;
  for (int p = 0; p < n_plans; ++p) {
    if (!plans[p]) return TACSL_ERR_NULL_ARG;
    for (int q = 0; q < p; ++q)
      if (plans[q] == plans[p]) return TACSL_ERR_STATE;
  }
  // a plan with a pose path reads each substep's object pose from the row the
  // path step writes
  std::vector<tacsl_state> st(states, states + (int64_t)n_steps * n_plans);
  for (int s = 0; s < n_steps; ++s)
    for (int p = 0; p < n_plans; ++p)
      if (paths && paths[p].poses) st[(int64_t)s * n_plans + p].obj_pose = paths[p].poses + (int64_t)s * 7 * plans[p]->n_env;
  for (int s = 0; s < n_steps; ++s)
    for (int p = 0; p < n_plans; ++p) {
      const int64_t k = (int64_t)s * n_plans + p;
      int rc = check_state(plans[p], st.data() + k);
      if (rc != TACSL_OK) return rc;
      rc = check_outputs(plans[p], outs + k);
      if (rc != TACSL_OK) return rc;
    }
  tacsl_graph g = new (std::nothrow) tacsl_graph_s();
  if (!g) return TACSL_ERR_ALLOC;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) {
    delete g;
    return TACSL_ERR_HIP;
  }
  int rc = TACSL_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) rc = TACSL_ERR_HIP;
  for (int s = 0; s < n_steps && rc == TACSL_OK; ++s)
    for (int p = 0; p < n_plans && rc == TACSL_OK; ++p) {
      const int64_t k = (int64_t)s * n_plans + p;
      if (paths && paths[p].poses && plans[p]->n_env > 0 &&
          tacsl::launch_pose_step(paths[p].pose0, paths[p].twist, s * paths[p].dt, plans[p]->n_env,
                                  paths[p].poses + (int64_t)s * 7 * plans[p]->n_env, cs) != hipSuccess)
        rc = TACSL_ERR_HIP;
      if (rc == TACSL_OK) rc = enqueue_forward(plans[p], st.data() + k, outs + k, cs, true);
    }
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &graph);
  if (rc == TACSL_OK && e != hipSuccess) rc = TACSL_ERR_HIP;
  if (rc == TACSL_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) rc = TACSL_ERR_HIP;
  (void)hipStreamDestroy(cs);
  if (rc != TACSL_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    delete g;
    return rc;
  }
  g->graph = graph;
  g->plans.assign(plans, plans + n_plans);
  for (tacsl_plan p : g->plans) p->live_graphs++;
  *out = g;
  return TACSL_OK;
}

int tacsl_graph_launch(tacsl_graph graph, hipStream_t stream) {
  const Range range("tacsl_graph_launch");
  if (!graph || !graph->exec) return TACSL_ERR_NULL_ARG;
  return hipGraphLaunch(graph->exec, stream) == hipSuccess ? TACSL_OK : TACSL_ERR_HIP;
}

int tacsl_graph_destroy(tacsl_graph graph) {
  if (!graph) return TACSL_OK;
  if (graph->exec) (void)hipGraphExecDestroy(graph->exec);
  if (graph->graph) (void)hipGraphDestroy(graph->graph);
  for (tacsl_plan p : graph->plans) p->live_graphs--;
  delete graph;
  return TACSL_OK;
}

int tacsl_plan_timer_start(tacsl_plan plan, int32_t capacity) {
  if (!plan) return TACSL_ERR_NULL_ARG;
  if (capacity < 0) return TACSL_ERR_RANGE;
  plan->free_timer();
  for (int32_t k = 0; k < capacity; ++k) {
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) {
      plan->free_timer();
      return TACSL_ERR_HIP;
    }
    if (hipEventCreate(&b) != hipSuccess) {
      (void)hipEventDestroy(a);
      plan->free_timer();
      return TACSL_ERR_HIP;
    }
    plan->ev_start.push_back(a);
    plan->ev_stop.push_back(b);
  }
  return TACSL_OK;
}

int tacsl_plan_timer_read(tacsl_plan plan, int32_t max, int32_t* n, float* ms) {
  if (!plan || !n || (max > 0 && !ms)) return TACSL_ERR_NULL_ARG;
  const int32_t m = std::min(max, plan->timer_n);
  for (int32_t k = 0; k < m; ++k) {
    if (hipEventSynchronize(plan->ev_stop[k]) != hipSuccess) return TACSL_ERR_HIP;
    if (hipEventElapsedTime(ms + k, plan->ev_start[k], plan->ev_stop[k]) != hipSuccess) return TACSL_ERR_HIP;
  }
  *n = m;
  return TACSL_OK;
}

int tacsl_plan_destroy(tacsl_plan plan) {
  if (!plan) return TACSL_OK;
  if (plan->live_graphs > 0) return TACSL_ERR_STATE;
  (void)hipDeviceSynchronize();
  plan->free_all();
  delete plan;
  return TACSL_OK;
}

}  // extern "C"
