// Execution of function bodies: grouped MLP launches (one persistent kernel
// per layer, replayed from a captured hipGraph), batched stencil sweeps, and
// the tile-shape autotuner.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <fstream>
#include <sstream>

#include "internal.h"

namespace sage {

size_t in_elem_size(const sage_fn_desc& d) { return d.kind == SAGE_MLP_BF16 ? 2 : 4; }

uint64_t ro_bytes_for(const sage_fn_desc& d) {
  if (d.kind == SAGE_STENCIL7_F32) return (uint64_t)d.nx * d.ny * d.nz * 4;
  if (d.kind == SAGE_RELAX7_F32) return 0;
  return (uint64_t)d.layers * d.width * d.width * in_elem_size(d);
}

size_t in_bytes_for(const sage_fn_desc& d, uint32_t batch) {
  if (is_grid(d.kind)) return (size_t)batch * d.nx * d.ny * d.nz * 4;
  return (size_t)batch * d.width * in_elem_size(d);
}

size_t out_bytes_for(const sage_fn_desc& d, uint32_t batch) {
  if (is_grid(d.kind)) return (size_t)batch * d.nx * d.ny * d.nz * 4;
  return (size_t)batch * d.width * 4;
}

// ------------------------------------------------------------- tile shapes
struct TileShape {
  const char* name;
  uint32_t bm, bn, occupancy, threads;
  bool ranged;     // tiles dealt to XCDs in contiguous ranges (grid a multiple of 8)
  uint32_t kalign = 64;  // K must be a multiple of this
};
static const TileShape kShapes[] = {
    {"ggemm6p_bf16_256x256", 256, 256, 1, 512, true},  {"ggemm6_bf16_256x128", 256, 128, 1, 512, true},
    {"ggemm2_bf16_128x256", 128, 256, 1, 512, true},   {"ggemm_bf16_128x128", 128, 128, 2, 256, false},
    {"ggemm3_bf16_128x64", 128, 64, 1, 256, true},     {"ggemm_bf16_64x128", 64, 128, 2, 256, false},
    {"ggemm_bf16_32x128", 32, 128, 2, 256, false},     {"ggemm3g4_bf16_64x64", 64, 64, 1, 256, true, 128},
    {"ggemm3g4_bf16_32x64", 32, 64, 1, 128, true, 128}, {"ggemm3g4_bf16_16x64", 16, 64, 2, 64, true, 128},
    {"ggemm3t_bf16_32x32", 32, 32, 2, 128, true, 128},  {"ggemm3t_bf16_16x32", 16, 32, 3, 64, true, 128},
    {"ggemm3t_bf16_16x16", 16, 16, 4, 64, true, 128},
};

static bool fits(const TileShape& ts, uint32_t W) { return W % ts.bn == 0 && W % ts.kalign == 0; }

static const TileShape& shape_of(const std::string& name) {
  for (const auto& s : kShapes)
    if (name == s.name) return s;
  fail(SAGE_EINVAL, "unknown tile shape %s", name.c_str());
}

// ------------------------------------------------------------------ flights
// meta buffer: [main header | main groups][tail header | tail groups][input row
// table][output row table]
constexpr uint32_t kMaxGroups = 256;
constexpr size_t kMetaGroupsOff = 16;
constexpr size_t kMetaTailOff = kMetaGroupsOff + kMaxGroups * sizeof(GemmGroup);
constexpr size_t kMetaTabOff = 2 * kMetaTailOff;
constexpr uint32_t kXcdCount = 8;

struct MlpPlan {
  const TileShape* main = nullptr;
  const TileShape* tail = nullptr;   // thin shape of the split-off ragged row tiles
  std::vector<uint8_t> split;        // per group: its ragged last row tile runs in the tail launch
  double cost_ms = 0;                // predicted layer time
};
uint32_t shape_grid(const Ctx& c, const TileShape& ts);
MlpPlan plan_mlp(Ctx& c, uint32_t W, const std::vector<uint32_t>& m, bool may_tune = true);

void flights_init(Ctx& c) {
  c.flights.resize(std::max<uint32_t>(1, c.cfg.inflight_groups));
  for (Flight& F : c.flights) {
    HIPX(hipStreamCreateWithFlags(&F.s, hipStreamNonBlocking));
    HIPX(hipEventCreateWithFlags(&F.done, hipEventDisableTiming));
  }
}

static void drop_graphs(Flight& F) {
  for (auto& kv : F.graphs) (void)hipGraphExecDestroy(kv.second);
  F.graphs.clear();
}

void flights_drop_graphs(Ctx& c) {
  for (size_t i = 0; i < c.flights.size(); i++) {
    finish_flight(c, (int)i);
    drop_graphs(c.flights[i]);
  }
}

void flights_destroy(Ctx& c) {
  for (Flight& F : c.flights) {
    (void)hipStreamSynchronize(F.s);
    drop_graphs(F);
    (void)hipFree(F.d_meta);
    (void)hipHostFree(F.h_meta);
    (void)hipFree(F.ws);
    (void)hipFree(F.d_in);
    (void)hipHostFree(F.h_in);
    (void)hipFree(F.d_out);
    (void)hipHostFree(F.h_out);
    (void)hipEventDestroy(F.done);
    (void)hipStreamDestroy(F.s);
  }
  c.flights.clear();
}

static size_t grow(size_t need) {
  size_t cap = 1u << 20;
  while (cap < need) cap <<= 1;
  return cap;
}

// Device/pinned buffer pair grown to at least `need` bytes; returns true
// when it moved (graphs holding the old address must be re-captured).
static bool ensure(uint8_t** d, uint8_t** h, size_t* cap, size_t need) {
  if (*cap >= need) return false;
  const size_t n = grow(need);
  if (*d) HIPX(hipFree(*d));
  if (h && *h) HIPX(hipHostFree(*h));
  *d = nullptr;
  HIPX(hipMalloc((void**)d, n));
  if (h) HIPX(hipHostMalloc((void**)h, n, hipHostMallocDefault));
  *cap = n;
  return true;
}

static int take_flight(Ctx& c, int want) {
  const int f = want >= 0 ? want : (int)(c.next_flight++ % c.flights.size());
  if (c.flights[f].busy) finish_flight(c, f);
  return f;
}

int free_flight(Ctx& c) {
  for (size_t i = 0; i < c.flights.size(); i++)
    if (!c.flights[i].busy) return (int)i;
  return -1;
}

void finish_flight(Ctx& c, int f) {
  Flight& F = c.flights[f];
  if (!F.busy) return;
  HIPX(hipEventSynchronize(F.done));
  std::vector<HostCopy> out;
  out.reserve(F.deliver.size());
  for (auto& d : F.deliver) out.push_back({(uint8_t*)d.first, F.h_out + d.second.first, d.second.second});
  copy_parallel(c, out);
  F.deliver.clear();
  F.busy = false;
  c.timer.collect();
}

static void launch_kernel(hipFunction_t k, uint32_t grid, uint32_t threads, hipStream_t s, const GemmHdr* hdr,
                          const GemmGroup* groups, const LayerArgs& la) {
  const GemmHdr* h = hdr;
  const GemmGroup* g = groups;
  LayerArgs a = la;
  void* params[] = {&h, &g, &a};
  HIPX(hipModuleLaunchKernel(k, grid, 1, 1, threads, 1, 1, 0, s, params, nullptr));
}

// The FP32 layer also takes its only group by value (wtab1 null: read the
// groups from the header as the BF16 kernels do).
static void launch_f32(hipFunction_t k, uint32_t grid, uint32_t threads, hipStream_t s, const GemmHdr* hdr,
                       const GemmGroup* groups, const LayerArgs& la, const uint64_t* wtab1, uint32_t m1) {
  const GemmHdr* h = hdr;
  const GemmGroup* g = groups;
  LayerArgs a = la;
  const uint64_t* w = wtab1;
  uint32_t m = m1;
  void* params[] = {&h, &g, &a, &w, &m};
  HIPX(hipModuleLaunchKernel(k, grid, 1, 1, threads, 1, 1, 0, s, params, nullptr));
}

// ---------------------------------------------------------------- MLP group
// All calls share kind, width and depth.  Rows of the calls of one weight
// table (one function, or one private copy) are packed into one group; the
// launch covers all groups with one tile list.  Layer 0 reads the inputs
// through a row table, the last layer writes the outputs through another;
// hidden layers ping-pong in the flight's workspace.
//
// A BF16 layer may run as two launches: the main tile shape over every
// group's full row tiles, and a thin tile shape over the ragged last row
// tiles of some groups, when that removes a nearly empty last wave of large
// tiles (see plan_mlp).  Both cover disjoint outputs of the same row space.
//
// With `ext` the metadata and the activations live in the caller's buffers
// instead of the flight's (nothing is allocated): device I/O only, eager
// launches (no graph), no autotuning, no kernel timing.
int launch_mlp_group(Ctx& c, const std::vector<Call>& calls, uint32_t io, int flight, const ExtScratch* ext) {
  const sage_fn_desc& d = calls[0].inv->fn->d;
  const uint32_t W = d.width, L = d.layers;
  const bool bf16 = d.kind == SAGE_MLP_BF16;
  const size_t es_in = bf16 ? 2 : 4, es_act = es_in;

  // groups by weight table, first-appearance order
  std::vector<const uint64_t*> tabs;
  std::vector<std::vector<size_t>> members;
  for (size_t i = 0; i < calls.size(); i++) {
    const uint64_t* t = calls[i].inv->table();
    size_t g = 0;
    while (g < tabs.size() && tabs[g] != t) g++;
    if (g == tabs.size()) {
      tabs.push_back(t);
      members.emplace_back();
    }
    members[g].push_back(i);
  }
  if (tabs.size() > kMaxGroups) fail(SAGE_EINVAL, "more than %u weight tables in one launch", kMaxGroups);
  uint32_t M = 0;
  std::vector<uint32_t> gm(tabs.size(), 0);
  for (size_t g = 0; g < tabs.size(); g++)
    for (size_t i : members[g]) gm[g] += calls[i].inv->batch;
  for (uint32_t m : gm) M += m;

  const bool host_in = !(io & SAGE_IO_DEVICE_IN), host_out = !(io & SAGE_IO_DEVICE_OUT);
  if (ext) {
    if (host_in || host_out) fail(SAGE_EINVAL, "caller-scratch launches take device I/O only");
    if (kMetaTabOff + (size_t)M * 16 > ext->meta_cap || 2 * (size_t)M * W * es_act > ext->ws_cap)
      fail(SAGE_EINVAL, "%u rows of width %u exceed the scratch buffer", M, W);
  }
  MlpPlan plan;
  if (bf16) plan = plan_mlp(c, W, gm, ext == nullptr);

  const int fi = take_flight(c, flight);
  Flight& F = c.flights[fi];
  uint8_t *d_meta, *h_meta, *ws;
  size_t meta_cap, ws_cap;
  if (ext) {
    d_meta = ext->d_meta;
    h_meta = ext->h_meta;
    meta_cap = ext->meta_cap;
    ws = ext->ws;
    ws_cap = ext->ws_cap;
  } else {
    bool moved = false;
    moved |= ensure(&F.d_meta, &F.h_meta, &F.meta_cap, kMetaTabOff + (size_t)M * 16);
    moved |= ensure(&F.ws, nullptr, &F.ws_cap, 2 * (size_t)M * W * es_act);
    // graphs hold meta/workspace addresses and the row capacity
    if (moved) drop_graphs(F);
    if (host_in) ensure(&F.d_in, &F.h_in, &F.in_cap, (size_t)M * W * es_in);
    if (host_out) ensure(&F.d_out, &F.h_out, &F.out_cap, (size_t)M * W * 4);
    d_meta = F.d_meta;
    h_meta = F.h_meta;
    meta_cap = F.meta_cap;
    ws = F.ws;
    ws_cap = F.ws_cap;
  }
  const size_t rows_cap = (meta_cap - kMetaTabOff) / 16;

  GemmHdr* hdr = reinterpret_cast<GemmHdr*>(h_meta);
  GemmGroup* grp = reinterpret_cast<GemmGroup*>(h_meta + kMetaGroupsOff);
  GemmHdr* thdr = reinterpret_cast<GemmHdr*>(h_meta + kMetaTailOff);
  GemmGroup* tgrp = reinterpret_cast<GemmGroup*>(h_meta + kMetaTailOff + kMetaGroupsOff);
  uint64_t* in_tab = reinterpret_cast<uint64_t*>(h_meta + kMetaTabOff);
  uint64_t* out_tab = in_tab + rows_cap;
  uint32_t row = 0, tiles = 0, ttiles = 0, ng = 0, nt = 0;
  F.deliver.clear();
  std::vector<HostCopy> in_copies;  // host inputs into the pinned staging, copied after the loop
  for (size_t g = 0; g < tabs.size(); g++) {
    const uint32_t row0 = row;
    for (size_t i : members[g]) {
      const Call& cl = calls[i];
      const uint32_t b = cl.inv->batch;
      for (uint32_t r = 0; r < b; r++) {
        const uint32_t R = row + r;
        in_tab[R] = host_in ? (uint64_t)(F.d_in + (size_t)R * W * es_in)
                            : (uint64_t)((const uint8_t*)cl.in + (size_t)r * W * es_in);
        out_tab[R] = host_out ? (uint64_t)(F.d_out + (size_t)R * W * 4)
                              : (uint64_t)((uint8_t*)cl.out + (size_t)r * W * 4);
      }
      if (host_in) in_copies.push_back({F.h_in + (size_t)row * W * es_in, (const uint8_t*)cl.in, (size_t)b * W * es_in});
      if (host_out) F.deliver.push_back({cl.out, {(size_t)row * W * 4, (size_t)b * W * 4}});
      row += b;
    }
    const uint32_t m = gm[g];
    if (!bf16) {
      grp[ng++] = GemmGroup{(uint64_t)tabs[g], m, row0, tiles, 0};
      tiles += W / c.f32_cols;
      continue;
    }
    const uint32_t part = plan.tail && plan.split[g] ? m % plan.main->bm : 0;
    if (m - part) {
      grp[ng++] = GemmGroup{(uint64_t)tabs[g], m - part, row0, tiles, 0};
      tiles += ((m - part + plan.main->bm - 1) / plan.main->bm) * (W / plan.main->bn);
    }
    if (part) {
      tgrp[nt++] = GemmGroup{(uint64_t)tabs[g], part, row0 + (m - part), ttiles, 0};
      ttiles += ((part + plan.tail->bm - 1) / plan.tail->bm) * (W / plan.tail->bn);
    }
  }
  copy_parallel(c, in_copies);
  *hdr = GemmHdr{ng, tiles, M, 0};
  *thdr = GemmHdr{nt, ttiles, M, 0};
  const bool split = nt > 0;
  const TileShape* ms = bf16 ? plan.main : nullptr;
  const std::string kname = bf16 ? ms->name : c.f32_cols == 4 ? "mlp_f32_layer" : "mlp_f32_layer_c8";
  c.last_launch = kname + ":" + std::to_string(tiles);
  if (split) c.last_launch += std::string("+") + plan.tail->name + ":" + std::to_string(ttiles);

  hipStream_t s = F.s;
  // Readiness gate (the kernel executor's check).  A function whose
  // progressive reload is still landing is gated layer by layer below; any
  // other waits for its data, and for the progressive reloads in flight if
  // one of them fills a class it shares.
  std::vector<Fn*> gated, seen;
  bool fed = false;
  for (const Call& cl : calls) {
    Fn* fn = cl.inv->fn;
    if (std::find(seen.begin(), seen.end(), fn) != seen.end()) continue;
    seen.push_back(fn);
    if (reload_landing(c, *fn)) {
      gated.push_back(fn);
    } else {
      HIPX(hipStreamWaitEvent(s, fn->ready, 0));
      fed = fed || reload_feeds(c, *fn);
    }
  }
  if (fed) HIPX(hipStreamWaitEvent(s, c.reload_done, 0));
  HIPX(hipMemcpyAsync(d_meta, h_meta, kMetaGroupsOff + ng * sizeof(GemmGroup), hipMemcpyHostToDevice, s));
  if (split)
    HIPX(hipMemcpyAsync(d_meta + kMetaTailOff, h_meta + kMetaTailOff, kMetaGroupsOff + nt * sizeof(GemmGroup),
                        hipMemcpyHostToDevice, s));
  HIPX(hipMemcpyAsync(d_meta + kMetaTabOff, in_tab, (size_t)M * 8, hipMemcpyHostToDevice, s));
  HIPX(hipMemcpyAsync(d_meta + kMetaTabOff + rows_cap * 8, out_tab, (size_t)M * 8, hipMemcpyHostToDevice, s));
  if (host_in) HIPX(hipMemcpyAsync(F.d_in, F.h_in, (size_t)M * W * es_in, hipMemcpyHostToDevice, s));

  Module* mod = calls[0].inv->fn->mod;
  hipFunction_t kfn = mod->get(kname.c_str());
  hipFunction_t tfn = split ? mod->get(plan.tail->name) : nullptr;
  // the FP32 layer: one workgroup per tile up to four per CU (grid-stride
  // beyond), so that a few-row launch does not dispatch idle workgroups
  const uint32_t grid = bf16 ? shape_grid(c, *ms) : std::max<uint32_t>(1, std::min<uint32_t>(tiles, c.cus * 4));
  const uint32_t threads = bf16 ? ms->threads : 256;
  const uint32_t tgrid = split ? shape_grid(c, *plan.tail) : 0, tthreads = split ? plan.tail->threads : 0;
  const GemmHdr* d_hdr = reinterpret_cast<const GemmHdr*>(d_meta);
  const GemmGroup* d_grp = reinterpret_cast<const GemmGroup*>(d_meta + kMetaGroupsOff);
  const GemmHdr* d_thdr = reinterpret_cast<const GemmHdr*>(d_meta + kMetaTailOff);
  const GemmGroup* d_tgrp = reinterpret_cast<const GemmGroup*>(d_meta + kMetaTailOff + kMetaGroupsOff);
  const uint64_t* d_in_tab = reinterpret_cast<const uint64_t*>(d_meta + kMetaTabOff);
  const uint64_t* d_out_tab = d_in_tab + rows_cap;
  const size_t half = ws_cap / 2;
  auto layer_args = [&](uint32_t l) {
    LayerArgs la{};
    la.a_tab = l == 0 ? d_in_tab : nullptr;
    la.a_base = ws + ((l + 1) % 2) * half;
    la.c_tab = l == L - 1 ? d_out_tab : nullptr;
    la.c_base = ws + (l % 2) * half;
    la.w_off = (uint64_t)l * W * W * es_in;
    la.N = W;
    la.K = W;
    la.flags = (l + 1 < L ? kRelu : 0u) | (l + 1 == L ? kOutF32 : 0u);
    return la;
  };
  // a one-function FP32 launch passes its group by value; a graph would
  // keep those arguments, so such launches are not captured
  const bool f32_one = !bf16 && ng == 1;
  const uint64_t* one_tab = f32_one ? reinterpret_cast<const uint64_t*>(grp[0].wtab) : nullptr;
  const uint32_t one_m = f32_one ? grp[0].m : 0;
  auto layers = [&](hipStream_t st) {
    for (uint32_t l = 0; l < L; l++) {
      for (Fn* g : gated) HIPX(hipStreamWaitEvent(st, g->seg[l], 0));
      const LayerArgs la = layer_args(l);
      if (!bf16) launch_f32(kfn, grid, threads, st, d_hdr, d_grp, la, one_tab, one_m);
      else if (tiles) launch_kernel(kfn, grid, threads, st, d_hdr, d_grp, la);
      if (split) launch_kernel(tfn, tgrid, tthreads, st, d_thdr, d_tgrp, la);
    }
  };
  const char* tname = bf16 ? "ggemm_bf16" : "mlp_f32";
  // a gated launch's span includes copy waits: it is not timed, nor captured
  const int tok = gated.empty() && !ext ? c.timer.start(tname, s, L) : -1;
  if (c.cfg.batch && gated.empty() && !ext && !f32_one) {
    // the FP32 layer's grid follows its tile count: part of the key
    const GraphKey key{kname + (split ? std::string("+") + plan.tail->name : std::string()) + (tiles ? "" : "/tail") +
                           (bf16 ? std::string() : "/" + std::to_string(grid)),
                       L, W};
    auto it = F.graphs.find(key);
    if (it == F.graphs.end()) {
      hipStream_t cap = s;
      HIPX(hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed));
      layers(cap);
      hipGraph_t g = nullptr;
      HIPX(hipStreamEndCapture(cap, &g));
      hipGraphExec_t ex = nullptr;
      HIPX(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
      HIPX(hipGraphDestroy(g));
      it = F.graphs.emplace(key, ex).first;
    }
    HIPX(hipGraphLaunch(it->second, s));
  } else {
    layers(s);
  }
  c.timer.stop(tok, s);
  if (host_out) HIPX(hipMemcpyAsync(F.h_out, F.d_out, (size_t)M * W * 4, hipMemcpyDeviceToHost, s));
  HIPX(hipEventRecord(F.done, s));
  F.busy = true;
  return fi;
}

// ------------------------------------------------------------ stencil group
// All calls share one coefficient table.  Every field of every call is
// swept together.  The sweeps run as passes of two (stencil7_fused2: u0 read
// and u2 written once per two sweeps), after one single sweep
// (stencil7_sweep2) when their number is odd; a pass's output goes to the
// call's output buffer on the last pass and alternates with a scratch field
// before it.
int launch_stencil_group(Ctx& c, const std::vector<Call>& calls, uint32_t io, int flight) {
  const sage_fn_desc& d = calls[0].inv->fn->d;
  const uint64_t cells = (uint64_t)d.nx * d.ny * d.nz, fbytes = cells * 4;
  const uint32_t S = d.sweeps;
  uint32_t nf = 0;
  for (const Call& cl : calls) nf += cl.inv->batch;
  const bool host_in = !(io & SAGE_IO_DEVICE_IN), host_out = !(io & SAGE_IO_DEVICE_OUT);

  const int fi = take_flight(c, flight);
  Flight& F = c.flights[fi];
  hipStream_t s = F.s;
  for (const Call& cl : calls) HIPX(hipStreamWaitEvent(s, cl.inv->fn->ready, 0));
  bool fed = false;
  for (const Call& cl : calls) fed = fed || reload_feeds(c, *cl.inv->fn);
  if (fed) HIPX(hipStreamWaitEvent(s, c.reload_done, 0));
  std::vector<uint32_t> pass;  // sweeps per pass
  if (c.stencil_fuse) {
    if (S % 2) pass.push_back(1);
    for (uint32_t i = 0; i < S / 2; i++) pass.push_back(2);
  } else {
    pass.assign(S, 1);
  }
  const uint32_t P = (uint32_t)pass.size();
  // the flight's captured MLP graphs hold the meta buffer's address and row
  // capacity: a move makes them stale
  if (ensure(&F.d_meta, &F.h_meta, &F.meta_cap, (size_t)std::max<uint32_t>(S, 1) * 2 * nf * 8)) drop_graphs(F);
  uint64_t* tab = reinterpret_cast<uint64_t*>(F.h_meta);
  F.deliver.clear();
  std::vector<std::pair<const uint8_t*, uint8_t*>> io_fields;  // (input, final output) per field
  uint32_t fidx = 0;
  for (const Call& cl : calls) {
    Inv& v = *cl.inv;
    const size_t bytes = (size_t)v.batch * fbytes;
    if (!v.ws) v.ws = c.cache.get(bytes);
    const uint8_t* in = (const uint8_t*)cl.in;
    uint8_t* out = (uint8_t*)cl.out;
    if (host_in) {
      if (!v.io_in) v.io_in = c.cache.get(bytes);
      HIPX(hipMemcpyAsync(v.io_in, cl.in, bytes, hipMemcpyHostToDevice, s));
      in = (const uint8_t*)v.io_in;
    }
    if (host_out) {
      if (!v.io_out) v.io_out = c.cache.get(bytes);
      out = (uint8_t*)v.io_out;
    }
    for (uint32_t b = 0; b < v.batch; b++) {
      const uint8_t* fin = in + b * fbytes;
      uint8_t* fout = out + b * fbytes;
      uint8_t* scratch = (uint8_t*)v.ws + b * fbytes;
      const uint8_t* r = fin;
      for (uint32_t k = 0; k < P; k++) {
        uint8_t* w = ((P - 1 - k) % 2 == 0) ? fout : scratch;
        tab[(size_t)k * 2 * nf + fidx] = (uint64_t)r;
        tab[(size_t)k * 2 * nf + nf + fidx] = (uint64_t)w;
        r = w;
      }
      io_fields.push_back({fin, fout});
      fidx++;
    }
  }
  // the coefficient grid's block table, or none: one constant coefficient
  const uint64_t* ctab = d.kind == SAGE_STENCIL7_F32 ? calls[0].inv->table() : nullptr;
  if (S == 0) {
    for (auto& p : io_fields) HIPX(hipMemcpyAsync(p.second, p.first, fbytes, hipMemcpyDeviceToDevice, s));
  } else {
    HIPX(hipMemcpyAsync(F.d_meta, F.h_meta, (size_t)P * 2 * nf * 8, hipMemcpyHostToDevice, s));
    Module* mod = calls[0].inv->fn->mod;
    hipFunction_t k1 = mod->get("stencil7_sweep2");
    hipFunction_t k2 = mod->get("stencil7_fused2");
    // the timer counts sweeps: a pass of two is two units of its time
    const int tok = c.timer.start("stencil7", s, S);
    for (uint32_t k = 0; k < P; k++) {
      const bool fused = pass[k] == 2;
      StencilArgs sa{};
      sa.ctab = ctab;
      sa.coef = d.coef;
      sa.nx = d.nx;
      sa.ny = d.ny;
      sa.nz = d.nz;
      sa.n_fields = nf;
      sa.tiles_x = (d.nx + kStencil2TX - 1) / kStencil2TX;
      const uint32_t rows = fused ? kStencil2TY - 2 : kStencil2TY;  // output rows per tile
      sa.tiles_y = (d.ny + rows - 1) / rows;
      sa.tiles_z = (d.nz + kStencil2TZ - 1) / kStencil2TZ;
      sa.spatial_tiles = sa.tiles_x * sa.tiles_y * sa.tiles_z;
      const uint64_t groups = (uint64_t)((sa.spatial_tiles + 7) / 8) * 8 * nf;
      if (groups > 0x7FFFFFFFull) fail(SAGE_EINVAL, "stencil launch too large");
      sa.src = reinterpret_cast<const uint64_t*>(F.d_meta) + (size_t)k * 2 * nf;
      sa.dst = sa.src + nf;
      void* params[] = {&sa};
      HIPX(hipModuleLaunchKernel(fused ? k2 : k1, (uint32_t)groups, 1, 1, 1024, 1, 1, 0, s, params, nullptr));
    }
    c.timer.stop(tok, s);
  }
  if (host_out) {
    for (const Call& cl : calls)
      HIPX(hipMemcpyAsync(cl.out, cl.inv->io_out, (size_t)cl.inv->batch * fbytes, hipMemcpyDeviceToHost, s));
  }
  HIPX(hipEventRecord(F.done, s));
  F.busy = true;
  return fi;
}

// ---------------------------------------------------------------- autotuner
// Each tile shape's time for one full wave of tiles (one tile per workgroup
// of its grid, K = width deep) is measured once per width on a synthetic
// layer.  A launch of T tiles then costs waves(T) full-wave times, where a
// ranged shape's waves are set by its largest XCD range.  All shapes give
// bit-identical results (same MFMA, same K order), so neither the choice
// nor a main/tail split changes any output.
uint32_t shape_grid(const Ctx& c, const TileShape& ts) {
  return std::max<uint32_t>(8, (uint32_t)c.cus * ts.occupancy / 8 * 8);
}

static uint64_t waves_of(const TileShape& ts, uint32_t grid, uint64_t tiles) {
  if (!tiles) return 0;
  if (!ts.ranged) return (tiles + grid - 1) / grid;
  const uint64_t per_range = (tiles + kXcdCount - 1) / kXcdCount, per_xcd = grid / kXcdCount;
  return (per_range + per_xcd - 1) / per_xcd;
}

static uint64_t tiles_of(const TileShape& ts, uint32_t W, uint32_t rows) {
  return (uint64_t)((rows + ts.bm - 1) / ts.bm) * (W / ts.bn);
}

static void tune_save(Ctx& c) {
  if (!c.cfg.tune_cache) return;
  std::ofstream o(c.cfg.tune_cache);
  for (auto& kv : c.tune) o << kv.first << " " << kv.second.kernel << " " << kv.second.ms << "\n";
}

void tune_load(Ctx& c) {
  if (!c.cfg.tune_cache) return;
  std::ifstream in(c.cfg.tune_cache);
  std::string key, k;
  double ms;
  while (in >> key >> k >> ms) {
    bool ok = false;
    for (const auto& s : kShapes) ok |= k == s.name;
    if (ok && ms > 0) c.tune[key] = TuneEntry{k, ms};
  }
}

static std::string tune_key(uint32_t width, const TileShape& ts) {
  return std::to_string(width) + ":" + ts.name;
}

// Full-wave time of every shape that divides `width`, measured on first use.
static void tune_width(Ctx& c, uint32_t width) {
  bool all = true;
  for (const auto& ts : kShapes)
    if (fits(ts, width)) all &= c.tune.count(tune_key(width, ts)) > 0;
  if (all) return;
  Module* mod = load_module(c, SAGE_MLP_BF16);
  uint32_t max_rows = 0;
  for (const auto& ts : kShapes) {
    if (!fits(ts, width)) continue;
    const uint32_t nt = width / ts.bn, grid = shape_grid(c, ts);
    max_rows = std::max(max_rows, ((grid + nt - 1) / nt) * ts.bm);
  }
  const size_t wbytes = (size_t)width * width * 2, nblk = (wbytes + kBlock - 1) / kBlock;
  uint8_t* w = (uint8_t*)c.cache.get(wbytes);
  uint8_t* a = (uint8_t*)c.cache.get((size_t)max_rows * width * 2);
  uint8_t* o = (uint8_t*)c.cache.get((size_t)max_rows * width * 2);
  uint8_t* meta = (uint8_t*)c.cache.get(4096 + nblk * 8);
  std::vector<uint64_t> tab(nblk);
  for (size_t b = 0; b < nblk; b++) tab[b] = (uint64_t)(w + b * kBlock);
  hipStream_t s = c.ctl;
  // small non-zero values (BF16 0x3C00 = 1/128), alternating sign in the
  // weights: data-dependent power stays closer to a real layer's
  HIPX(hipMemsetD32Async((hipDeviceptr_t)w, 0xBC003C00u, wbytes / 4, s));
  HIPX(hipMemsetD16Async((hipDeviceptr_t)a, 0x3C00, (size_t)max_rows * width, s));
  HIPX(hipMemcpyAsync(meta + 4096, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, s));
  HIPX(hipStreamSynchronize(s));
  hipEvent_t e0, e1;
  HIPX(hipEventCreate(&e0));
  HIPX(hipEventCreate(&e1));
  for (const auto& ts : kShapes) {
    if (!fits(ts, width) || c.tune.count(tune_key(width, ts))) continue;
    const uint32_t nt = width / ts.bn, grid = shape_grid(c, ts);
    const uint32_t rows = ((grid + nt - 1) / nt) * ts.bm;
    const uint64_t tiles = tiles_of(ts, width, rows);
    GemmHdr h{1, (uint32_t)tiles, rows, 0};
    GemmGroup g{(uint64_t)(meta + 4096), rows, 0, 0, 0};
    HIPX(hipMemcpyAsync(meta, &h, sizeof h, hipMemcpyHostToDevice, s));
    HIPX(hipMemcpyAsync(meta + 16, &g, sizeof g, hipMemcpyHostToDevice, s));
    HIPX(hipStreamSynchronize(s));
    LayerArgs la{};
    la.a_base = a;
    la.c_base = o;
    la.N = la.K = width;
    la.flags = kRelu;
    hipFunction_t k = mod->get(ts.name);
    auto run = [&] { launch_kernel(k, grid, ts.threads, s, (const GemmHdr*)meta, (const GemmGroup*)(meta + 16), la); };
    run();
    const int reps = 4;
    HIPX(hipEventRecord(e0, s));
    for (int r = 0; r < reps; r++) run();
    HIPX(hipEventRecord(e1, s));
    HIPX(hipEventSynchronize(e1));
    float ms = 0;
    HIPX(hipEventElapsedTime(&ms, e0, e1));
    c.tune[tune_key(width, ts)] = TuneEntry{ts.name, (double)ms / reps / (double)waves_of(ts, grid, tiles)};
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c.cache.put(w);
  c.cache.put(a);
  c.cache.put(o);
  c.cache.put(meta);
  tune_save(c);
}

// Gap between two dependent kernels of one stream, charged to a split plan.
constexpr double kLaunchGapMs = 0.004;

// Cheapest plan for groups of `m` rows under full-wave times `tune`
// ("width:shape" -> ms; shapes without an entry are not considered): one
// shape over all tiles, or a large shape over every group's row tiles except
// the ragged last tiles of the groups in `split`, which a thin shape covers
// in a second launch.  Candidate splits move the k smallest ragged tiles.
static MlpPlan plan_from(const std::map<std::string, TuneEntry>& tune, uint32_t cus, uint32_t W,
                         const std::vector<uint32_t>& m) {
  MlpPlan best;
  best.split.assign(m.size(), 0);
  auto grid_of = [&](const TileShape& ts) { return std::max<uint32_t>(8, cus * ts.occupancy / 8 * 8); };
  auto wave = [&](const TileShape& ts) -> double {
    auto it = tune.find(tune_key(W, ts));
    return it == tune.end() ? -1.0 : it->second.ms;
  };
  double best_cost = 1e300;
  std::vector<std::pair<uint32_t, size_t>> parts;  // (ragged rows, group)
  for (const auto& ts : kShapes) {
    if (!fits(ts, W) || wave(ts) < 0) continue;
    const uint32_t grid = grid_of(ts);
    uint64_t tiles = 0;
    parts.clear();
    for (size_t g = 0; g < m.size(); g++) {
      tiles += tiles_of(ts, W, m[g]);
      if (m[g] % ts.bm) parts.push_back({m[g] % ts.bm, g});
    }
    const double cost = waves_of(ts, grid, tiles) * wave(ts);
    if (cost < best_cost) {
      best_cost = cost;
      best.main = &ts;
      best.tail = nullptr;
      std::fill(best.split.begin(), best.split.end(), 0);
    }
    if (ts.bm < 128 || parts.empty()) continue;
    std::sort(parts.begin(), parts.end());
    const uint64_t per_part = W / ts.bn;
    for (const auto& tt : kShapes) {
      if (!fits(tt, W) || wave(tt) < 0 || tt.bm >= ts.bm || !tt.ranged) continue;
      const uint32_t tgrid = grid_of(tt);
      uint64_t ttiles = 0;
      for (size_t k = 1; k <= parts.size() && k <= 64; k++) {
        ttiles += tiles_of(tt, W, parts[k - 1].first);
        const uint64_t main_tiles = tiles - k * per_part;
        const double sc = waves_of(ts, grid, main_tiles) * wave(ts) + waves_of(tt, tgrid, ttiles) * wave(tt) +
                          kLaunchGapMs;
        if (sc < best_cost) {
          best_cost = sc;
          best.main = &ts;
          best.tail = &tt;
          std::fill(best.split.begin(), best.split.end(), 0);
          for (size_t i = 0; i < k; i++) best.split[parts[i].second] = 1;
        }
      }
    }
  }
  if (!best.main) fail(SAGE_EINVAL, "no tile shape fits width %u", W);
  best.cost_ms = best_cost;
  return best;
}

// may_tune = false: plan from the full-wave times already measured for W
// (none: the 128 x 128 shape, which fits every supported width); every
// shape gives the same bits, so only the speed depends on it.
MlpPlan plan_mlp(Ctx& c, uint32_t W, const std::vector<uint32_t>& m, bool may_tune) {
  MlpPlan best;
  best.split.assign(m.size(), 0);
  if (!c.force_tile.empty()) {
    const size_t plus = c.force_tile.find('+');
    best.main = &shape_of(c.force_tile.substr(0, plus));
    if (plus != std::string::npos) {
      best.tail = &shape_of(c.force_tile.substr(plus + 1));
      for (size_t g = 0; g < m.size(); g++) best.split[g] = m[g] % best.main->bm != 0;
    }
    for (const TileShape* t : {best.main, best.tail})
      if (t && !fits(*t, W)) fail(SAGE_EINVAL, "tile %s does not fit width %u", t->name, W);
    return best;
  }
  if (!may_tune) {
    bool any = false;
    for (const auto& ts : kShapes) any |= fits(ts, W) && c.tune.count(tune_key(W, ts)) > 0;
    if (!any) {
      best.main = &shape_of("ggemm_bf16_128x128");
      if (!fits(*best.main, W)) fail(SAGE_EINVAL, "tile %s does not fit width %u", best.main->name, W);
      return best;
    }
    return plan_from(c.tune, (uint32_t)c.cus, W, m);
  }
  tune_width(c, W);
  return plan_from(c.tune, (uint32_t)c.cus, W, m);
}

// "main:tiles[+tail:tiles] cost_ms" of the plan for `m` under `tune`.
std::string plan_describe(const std::map<std::string, TuneEntry>& tune, uint32_t cus, uint32_t W,
                          const std::vector<uint32_t>& m) {
  const MlpPlan p = plan_from(tune, cus, W, m);
  uint64_t tiles = 0, ttiles = 0;
  for (size_t g = 0; g < m.size(); g++) {
    const uint32_t part = p.tail && p.split[g] ? m[g] % p.main->bm : 0;
    tiles += tiles_of(*p.main, W, m[g] - part);
    if (part) ttiles += tiles_of(*p.tail, W, part);
  }
  std::string s = std::string(p.main->name) + ":" + std::to_string(tiles);
  if (ttiles) s += std::string("+") + p.tail->name + ":" + std::to_string(ttiles);
  char buf[64];
  std::snprintf(buf, sizeof buf, " %.6f", p.cost_ms);
  return s + buf;
}

std::string tune_key_for(uint32_t width, const std::string& shape) { return std::to_string(width) + ":" + shape; }

bool tile_shape_known(const std::string& name) {
  for (const auto& s : kShapes)
    if (name == s.name) return true;
  return false;
}

}  // namespace sage
