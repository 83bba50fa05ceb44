// Batched relaxation of many grids: one kernel launch per RK stage covers
// every grid that is still relaxing, so catalogs of configurations with
// uneven grid sizes fill the device even when each grid alone would not (the
// paper's "Multiple, Independent Patches" experiment used one stream per
// patch instead).
//
// Work lists in device memory hold (grid, x0 tile, x1 tile, phi chunk) items
// (and in the stage lists (grid, -1, k, 0) items for blocks of outer points);
// persistent kernels walk them and read per-grid arguments from descriptor
// tables. The launch sequence of one check interval (base slopes and rebase
// of the split-state form, 4 x K stage launches, residual, per-grid norms) is
// captured once in a HIP graph and replayed; when grids converge or switch
// from the single-precision phase to the FP64 finish, only the lists and their
// lengths in device memory change. The host reads back one norm per grid per
// check and applies each grid's own stop test.
//
// Grids small enough for the resident kernel (state on chip, one patch per
// compute unit) skip the stage lists: per check interval they run K whole
// RK4 steps in resident launches, several grids per launch where their patches
// fit on the device together (each grid with its own counters and exchange
// buffers). These launches are part of the captured interval; the graph is
// captured again when the set of resident grids changes.

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "hr_internal.h"

using namespace hr;

struct hr_batch {
  int n = 0;
  int order = 0;
  int device = 0;
  std::vector<hr_grid*> g;
  bool bound = false;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  size_t cap_stage = 0, cap_plane = 0, cap_reb = 0;
  StageArgs<double>* sa64 = nullptr;
  StageArgs<float>* sa32 = nullptr;
  ResidualArgs* ra = nullptr;
  BaseArgs* ba = nullptr;
  RebaseArgs* rb = nullptr;
  int4* it64 = nullptr;
  int4* it32 = nullptr;
  int4* itres = nullptr;
  int4* itbase = nullptr;
  int2* itreb = nullptr;
  int* counts = nullptr;  // stage FP64, stage FP32 split, residual, base, rebase
  int4* ranges = nullptr;
  double* partial = nullptr;
  double* out = nullptr;
  double* host_out = nullptr;
  int nblk_tile = 512;
  int nblk_flat = 2048;
  int cus = 256;
  hipGraphExec_t exec = nullptr;
  int exec_mode = -1;
  int exec_K = 0;
  // resident grids: device argument tables (FP64 state, split-form increment),
  // their host copies, the launches they form and the shared error word
  ResidentArgsT<double>* rt64 = nullptr;
  ResidentArgsT<float>* rt32 = nullptr;
  unsigned* rerr = nullptr;
  std::vector<ResidentArgsT<double>> h_rt64;
  std::vector<ResidentArgsT<float>> h_rt32;
  struct ResGroup {
    bool split;
    int first;   // first entry of the group in its table
    int n;       // grids in the launch
  };
  std::vector<ResGroup> groups;
  std::vector<int> groups_sig;  // grouping of the resident grids (grid ids, phases)
  std::vector<int> exec_sig;    // grouping captured in exec
};

namespace {

hr_status bfail(hr_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

#define HR_HIPB(call)                                                                 \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      return bfail(HR_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
  } while (0)

size_t up256(size_t x) { return (x + 255) / 256 * 256; }

int tiles0(const hr_grid* g) { return (g->d.N0 + kTileX - 1) / kTileX; }
int tiles1(const hr_grid* g) { return (g->d.N1 + kTileY - 1) / kTileY; }
// Stage-list items holding a grid's boundary work (the NG N1 N2 outer points,
// and the 2 zo P0 N2 points of stored z-face rows), one tile's worth of
// threads each.
int outer_items(const hr_grid* g) {
  const Dims& d = g->d;
  return (d.NG * d.N1 * d.N2 + 2 * d.zo * d.P0 * d.N2 + kTileX * kTileY - 1) / (kTileX * kTileY);
}

// An explicit phi-column configuration of a grid keeps its chunk in a batch.
bool explicit_chunk(const hr_grid* g) { return g->variant == 2 && g->chunk > 0; }

// The phi chunk of the other grids of a batch: the largest of 16, 8, 4, 2 planes
// (capped at each grid's N2) whose work list still holds an item per compute
// unit, else single planes. Longer chunks load each column's phi taps once for
// more planes; shorter ones give small batches more items to spread over the
// chip (swept over 1..7 grids of 64x64x8, 128x128x16 and 256x256x32).
int batch_chunk(const hr_batch* b) {
  for (int c = 16; c > 1; c /= 2) {
    long items = 0;
    for (int i = 0; i < b->n; ++i) {
      const hr_grid* g = b->g[i];
      const int ch = explicit_chunk(g) ? g->chunk : std::min(c, g->d.N2);
      items += (long)tiles0(g) * tiles1(g) * ((g->d.N2 + ch - 1) / ch);
    }
    if (items >= b->cus) return c;
  }
  return 1;
}

size_t batch_layout(hr_batch* b, char* base) {
  size_t off = 0;
  auto take = [&](size_t bytes) -> char* {
    char* p = base ? base + off : nullptr;
    off = up256(off + bytes);
    return p;
  };
  const size_t n = b->n;
  b->sa64 = (StageArgs<double>*)take(4 * n * sizeof(StageArgs<double>));
  b->sa32 = (StageArgs<float>*)take(4 * n * sizeof(StageArgs<float>));
  b->ra = (ResidualArgs*)take(n * sizeof(ResidualArgs));
  b->ba = (BaseArgs*)take(n * sizeof(BaseArgs));
  b->rb = (RebaseArgs*)take(n * sizeof(RebaseArgs));
  b->it64 = (int4*)take(b->cap_stage * sizeof(int4));
  b->it32 = (int4*)take(b->cap_stage * sizeof(int4));
  b->itres = (int4*)take(b->cap_plane * sizeof(int4));
  b->itbase = (int4*)take(b->cap_plane * sizeof(int4));
  b->itreb = (int2*)take(b->cap_reb * sizeof(int2));
  b->counts = (int*)take(8 * sizeof(int));
  b->ranges = (int4*)take(n * sizeof(int4));
  b->partial = (double*)take(b->cap_plane * sizeof(double));
  b->out = (double*)take(n * sizeof(double));
  b->rt64 = (ResidentArgsT<double>*)take(n * sizeof(ResidentArgsT<double>));
  b->rt32 = (ResidentArgsT<float>*)take(n * sizeof(ResidentArgsT<float>));
  b->rerr = (unsigned*)take(sizeof(unsigned));
  return off;
}

// Phase of one grid during a batched relaxation.
struct GridRun {
  int phase = 1;       // 0 split-state single precision, 1 FP64
  bool done = false;
  int why = 0;         // 0 step cap, 1 tolerance, 2 non-finite
  long steps = 0;
  long f32steps = 0;
  double last = NAN;
  double best = INFINITY;
  int stall = 0;
  double sw = 0.0;
  int chunk = 1;
  double eta = 0.0;
  double dt = 0.0;
};

hr_status capture(hr_batch* b, int mode, int K) {
  if (b->exec) {
    (void)hipGraphExecDestroy(b->exec);
    b->exec = nullptr;
  }
  HR_HIPB(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  auto ok = [&](hipError_t x) {
    if (e == hipSuccess && x != hipSuccess) e = x;
  };
  bool zf = false;   // a grid with stored z-face rows (SinhCylindrical)
  for (const hr_grid* g : b->g) zf = zf || g->d.zo > 0;
  if (mode & 1)
    ok(launch_batch_base(b->order, zf, b->ba, b->itbase, b->counts + 3, b->nblk_tile, b->stream));
  for (int k = 0; k < K; ++k)
    for (int s = 1; s <= 4; ++s) {
      if (mode & 4)
        ok(launch_batch_stage(b->order, s, true, zf, b->sa32, b->it32, b->counts + 1,
                              b->nblk_tile, b->stream));
      if (mode & 2)
        ok(launch_batch_stage(b->order, s, false, zf, b->sa64, b->it64, b->counts + 0,
                              b->nblk_tile, b->stream));
    }
  for (const hr_batch::ResGroup& rg : b->groups) {
    if (rg.split)
      ok(launch_resident_multi(b->order, b->rt32 + rg.first, b->h_rt32.data() + rg.first, rg.n,
                               b->stream));
    else
      ok(launch_resident_multi(b->order, b->rt64 + rg.first, b->h_rt64.data() + rg.first, rg.n,
                               b->stream));
  }
  if (mode & 1) ok(launch_batch_rebase(b->rb, b->itreb, b->counts + 4, b->nblk_flat, b->stream));
  ok(launch_batch_residual(b->order, zf, b->ra, b->itres, b->counts + 2, b->partial,
                           b->nblk_tile, b->stream));
  ok(launch_batch_finalize(b->ranges, b->partial, b->out, b->n, b->stream));
  hipGraph_t graph = nullptr;
  const hipError_t ee = hipStreamEndCapture(b->stream, &graph);
  if (e == hipSuccess) e = ee;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  if (graph) (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    b->exec = nullptr;
    return bfail(HR_EDEVICE, std::string("batch graph capture: ") + hipGetErrorString(e));
  }
  b->exec_mode = mode;
  b->exec_K = K;
  b->exec_sig = b->groups_sig;
  return HR_OK;
}

// Packs the running grids that run resident in their current phase into
// launches: first fit, largest grids first, into launches of one kernel
// instance whose patches all fit on the device at once. Builds the argument
// tables (K steps each, every grid's error flag the batch's word) and the
// grouping's signature; the tables are uploaded by the caller.
hr_status plan_resident(hr_batch* b, const std::vector<GridRun>& run, int K,
                        std::vector<bool>& resident) {
  struct Cand {
    int i;
    const hr_grid::ResPlan* p;
  };
  std::vector<Cand> cand;
  resident.assign(b->n, false);
  for (int i = 0; i < b->n; ++i) {
    if (run[i].done) continue;
    const hr_grid::ResPlan* p = batch_resident_part(b->g[i], run[i].phase == 0);
    if (p) cand.push_back({i, p});
  }
  std::stable_sort(cand.begin(), cand.end(),
                   [](const Cand& x, const Cand& y) { return x.p->blocks() > y.p->blocks(); });
  struct Open {
    bool split;
    const void* key;
    int ry, N2, blocks;
    size_t lds;
    std::vector<Cand> members;
  };
  std::vector<Open> open;
  for (const Cand& c : cand) {
    const hr_grid* g = b->g[c.i];
    const bool split = run[c.i].phase == 0;
    const void* key = resident_kernel_key(b->order, g->d.N2, split, c.p->ry);
    if (!key) continue;
    const size_t lds = resident_lds_bytes(g->d, split ? sizeof(float) : sizeof(double), c.p->ry);
    bool placed = false;
    for (Open& o : open) {
      if (o.split != split || o.key != key) continue;
      const size_t l = std::max(o.lds, lds);
      const int cap = resident_multi_capacity(b->order, o.N2, split, o.ry, l);
      if (o.blocks + c.p->blocks() > std::min(cap, kResMaxBlocks)) continue;
      o.lds = l;
      o.blocks += c.p->blocks();
      o.members.push_back(c);
      placed = true;
      break;
    }
    if (!placed) {
      const int cap = resident_multi_capacity(b->order, g->d.N2, split, c.p->ry, lds);
      if (c.p->blocks() > std::min(cap, kResMaxBlocks)) continue;  // stays on the stage lists
      open.push_back({split, key, c.p->ry, g->d.N2, c.p->blocks(), lds, {c}});
    }
  }
  b->groups.clear();
  b->h_rt64.clear();
  b->h_rt32.clear();
  b->groups_sig.clear();
  for (const Open& o : open) {
    hr_batch::ResGroup rg{o.split, o.split ? (int)b->h_rt32.size() : (int)b->h_rt64.size(),
                          (int)o.members.size()};
    int block0 = 0;
    b->groups_sig.push_back(o.split ? -2 : -1);
    for (const Cand& c : o.members) {
      hr_grid* g = b->g[c.i];
      resident[c.i] = true;
      b->groups_sig.push_back(c.i);
      b->groups_sig.push_back(c.p == &g->res[0] ? 8 : 4);
      if (o.split) {
        ResidentArgsT<float> a =
            resident_args_split_part(g, c.p, (float)run[c.i].eta, (float)run[c.i].dt, K);
        a.block0 = block0;
        a.err = b->rerr;
        b->h_rt32.push_back(a);
      } else {
        ResidentArgsT<double> a = resident_args_part(g, c.p, run[c.i].eta, run[c.i].dt, K);
        a.block0 = block0;
        a.err = b->rerr;
        b->h_rt64.push_back(a);
      }
      block0 += c.p->blocks();
    }
    b->groups.push_back(rg);
  }
  return HR_OK;
}

// Rebuilds and uploads the work lists (and the resident launches) for the
// grids still relaxing.
hr_status upload_lists(hr_batch* b, const std::vector<GridRun>& run, int K, int* mode) {
  std::vector<int4> l64, l32, lres, lbase;
  std::vector<int2> lreb;
  std::vector<int4> rng(b->n);
  std::vector<bool> resident;
  hr_status pst = plan_resident(b, run, K, resident);
  if (pst != HR_OK) return pst;
  *mode = 0;
  for (int i = 0; i < b->n; ++i) {
    const hr_grid* g = b->g[i];
    const int t0 = tiles0(g), t1 = tiles1(g), N2 = g->d.N2;
    rng[i] = make_int4((int)lres.size(), 0, g->d.nint, 0);
    if (run[i].done) continue;
    const int nch = (N2 + run[i].chunk - 1) / run[i].chunk;
    std::vector<int4>& ls = run[i].phase == 0 ? l32 : l64;
    // mode bits: 1 split-form grids (base slopes and rebase), 2 FP64 stage
    // items, 4 split-form stage items, 8 resident launches
    if (run[i].phase == 0) *mode |= 1;
    *mode |= resident[i] ? 8 : run[i].phase == 0 ? 4 : 2;
    if (!resident[i]) {
      for (int z = 0; z < nch; ++z)
        for (int y = 0; y < t1; ++y)
          for (int x = 0; x < t0; ++x) ls.push_back(make_int4(i, x, y, z));
      // the grid's boundary points (xx0 face, z-face rows), items of their own
      for (int k = 0; k < outer_items(g); ++k) ls.push_back(make_int4(i, -1, k, 0));
    }
    for (int z = 0; z < N2; ++z)
      for (int y = 0; y < t1; ++y)
        for (int x = 0; x < t0; ++x) {
          lres.push_back(make_int4(i, x, y, z));
          if (run[i].phase == 0) lbase.push_back(make_int4(i, x, y, z));
        }
    rng[i].y = (int)lres.size() - rng[i].x;
    if (run[i].phase == 0) {
      const int nb = (int)((g->G + kBlock - 1) / kBlock);
      for (int k = 0; k < nb; ++k) lreb.push_back(make_int2(i, k));
    }
  }
  const int cnt[8] = {(int)l64.size(), (int)l32.size(), (int)lres.size(), (int)lbase.size(),
                      (int)lreb.size(), 0, 0, 0};
  if (l64.size() > b->cap_stage || l32.size() > b->cap_stage || lres.size() > b->cap_plane ||
      lreb.size() > b->cap_reb)
    return bfail(HR_EINVAL, "batch work list exceeds its capacity");
  if (!l64.empty())
    HR_HIPB(hipMemcpyAsync(b->it64, l64.data(), l64.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
  if (!l32.empty())
    HR_HIPB(hipMemcpyAsync(b->it32, l32.data(), l32.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
  if (!lres.empty())
    HR_HIPB(hipMemcpyAsync(b->itres, lres.data(), lres.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
  if (!lbase.empty())
    HR_HIPB(hipMemcpyAsync(b->itbase, lbase.data(), lbase.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
  if (!lreb.empty())
    HR_HIPB(hipMemcpyAsync(b->itreb, lreb.data(), lreb.size() * sizeof(int2), hipMemcpyHostToDevice, b->stream));
  HR_HIPB(hipMemcpyAsync(b->counts, cnt, sizeof(cnt), hipMemcpyHostToDevice, b->stream));
  HR_HIPB(hipMemcpyAsync(b->ranges, rng.data(), rng.size() * sizeof(int4), hipMemcpyHostToDevice, b->stream));
  if (!b->h_rt64.empty())
    HR_HIPB(hipMemcpyAsync(b->rt64, b->h_rt64.data(), b->h_rt64.size() * sizeof(b->h_rt64[0]),
                           hipMemcpyHostToDevice, b->stream));
  if (!b->h_rt32.empty())
    HR_HIPB(hipMemcpyAsync(b->rt32, b->h_rt32.data(), b->h_rt32.size() * sizeof(b->h_rt32[0]),
                           hipMemcpyHostToDevice, b->stream));
  HR_HIPB(hipStreamSynchronize(b->stream));
  return HR_OK;
}

}  // namespace

extern "C" {

hr_status hr_batch_create(int n, hr_grid* const* grids, hr_batch** out) {
  if (!out) return bfail(HR_EINVAL, "null output pointer");
  *out = nullptr;
  if (n < 1 || !grids) return bfail(HR_EINVAL, "need at least one grid");
  hr_batch* b = new (std::nothrow) hr_batch();
  if (!b) return bfail(HR_ENOMEM, "host allocation failed");
  b->n = n;
  b->g.assign(grids, grids + n);
  for (int i = 0; i < n; ++i) {
    hr_grid* g = grids[i];
    if (!g || !g->bound) {
      delete b;
      return bfail(HR_ESTATE, "every grid must be bound before batching");
    }
    for (int j = 0; j < i; ++j)
      if (grids[j] == g) {
        delete b;
        return bfail(HR_EINVAL, "a grid appears twice in the batch");
      }
    if (g->d.cart) {
      delete b;
      return bfail(HR_EINVAL, "Cartesian grids are not batched (relax them one by one)");
    }
    if (i == 0) {
      b->order = g->fd_order;
      b->device = g->device;
    } else if (g->fd_order != b->order || g->device != b->device) {
      delete b;
      return bfail(HR_EINVAL, "batched grids need the same fd_order and device");
    }
    const size_t tp = (size_t)tiles0(g) * tiles1(g) * g->d.N2;
    b->cap_stage += tp + outer_items(g);
    b->cap_plane += tp;
    b->cap_reb += (g->G + kBlock - 1) / kBlock;
  }
  *out = b;
  return HR_OK;
}

size_t hr_batch_workspace_bytes(const hr_batch* b) {
  if (!b) return 0;
  return batch_layout(const_cast<hr_batch*>(b), nullptr);
}

hr_status hr_batch_bind(hr_batch* b, void* dev_ptr, size_t bytes, void* hip_stream) {
  if (!b) return bfail(HR_EINVAL, "null batch");
  if (b->bound) return bfail(HR_ESTATE, "batch already bound");
  if (!dev_ptr || ((uintptr_t)dev_ptr % 256) != 0)
    return bfail(HR_EINVAL, "workspace pointer must be non-null and 256-byte aligned");
  if (bytes < batch_layout(b, nullptr)) return bfail(HR_ENOMEM, "workspace too small");
  HR_HIPB(hipSetDevice(b->device));
  if (hip_stream) {
    b->stream = (hipStream_t)hip_stream;
  } else {
    HR_HIPB(hipStreamCreate(&b->stream));
    b->own_stream = true;
  }
  // one norm per grid, then the resident launches' error word
  HR_HIPB(hipHostMalloc((void**)&b->host_out, (b->n + 1) * sizeof(double), hipHostMallocDefault));
  batch_layout(b, (char*)dev_ptr);
  int cus = 0;
  HR_HIPB(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device));
  b->nblk_tile = 2 * cus;
  b->nblk_flat = 8 * cus;
  b->cus = cus;
  b->bound = true;
  return HR_OK;
}

void hr_batch_destroy(hr_batch* b) {
  if (!b) return;
  if (b->bound) {
    (void)hipSetDevice(b->device);
    (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->host_out) (void)hipHostFree(b->host_out);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
  }
  delete b;
}

hr_status hr_batch_relax(hr_batch* b, const double* eta, const double* c, long n_steps,
                         double tol, int check_every, hr_precision prec,
                         hr_relax_report* reps) {
  if (!b) return bfail(HR_EINVAL, "null batch");
  if (!b->bound) return bfail(HR_ESTATE, "batch has no bound workspace");
  if (!eta || !c) return bfail(HR_EINVAL, "eta and c arrays are required");
  if (n_steps < 0 || check_every <= 0) return bfail(HR_EINVAL, "need n_steps >= 0, check_every > 0");
  if (prec != HR_FP64 && prec != HR_FP32_FP64FINISH)
    return bfail(HR_EINVAL, "batched precision must be HR_FP64 or HR_FP32_FP64FINISH");
  for (int i = 0; i < b->n; ++i) {
    if (!b->g[i]->have_sources) return bfail(HR_ESTATE, "punctures not set on a batched grid");
    if (b->g[i]->norm != 0)
      return bfail(HR_EINVAL, "batched relaxation uses the point norm (hr_set_residual_norm)");
    if (!(eta[i] > 0) || !(c[i] > 0) || !std::isfinite(eta[i]) || !std::isfinite(c[i]))
      return bfail(HR_EINVAL, "eta and c must be finite and > 0");
  }
  HR_HIPB(hipSetDevice(b->device));
  HR_HIPB(hipDeviceSynchronize());
  const int K = check_every;
  std::vector<GridRun> run(b->n);
  std::vector<StageArgs<double>> h64(4 * (size_t)b->n);
  std::vector<StageArgs<float>> h32(4 * (size_t)b->n);
  std::vector<ResidualArgs> hra(b->n);
  std::vector<BaseArgs> hba(b->n);
  std::vector<RebaseArgs> hrb(b->n);
  const int bchunk = batch_chunk(b);
  for (int i = 0; i < b->n; ++i) {
    hr_grid* g = b->g[i];
    hr_status st = load_kappa(g, c[i]);
    if (st != HR_OK) return st;
    const double dt = g->prm.cfl * g->tab.ds_g;
    const int chunk = explicit_chunk(g) ? g->chunk : std::min(bchunk, g->d.N2);
    run[i].chunk = chunk;
    run[i].eta = eta[i];
    run[i].dt = dt;
    run[i].phase = prec == HR_FP32_FP64FINISH ? 0 : 1;
    run[i].sw = g->sw_residual > 0 ? g->sw_residual : (tol > 0 ? 10.0 * tol : 0.0);
    for (int s = 1; s <= 4; ++s) {
      StageArgs<double> a = stage_args<double>(g, g->f64, s, eta[i], dt);
      a.variant = 2;
      a.chunk = chunk;
      h64[4 * i + s - 1] = a;
      StageArgs<float> f = stage_args<float>(g, g->f32, s, (float)eta[i], (float)dt, true);
      f.variant = 2;
      f.chunk = chunk;
      h32[4 * i + s - 1] = f;
    }
    hra[i] = ResidualArgs{g->d, g->f64.un, g->f64.psi, g->f64.ssrc, g->f64.fac, nullptr, nullptr};
    BaseArgs ba{};
    ba.d = g->d;
    ba.u = g->f64.un;
    ba.v = g->f64.vn;
    ba.psi = g->f64.psi;
    ba.ssrc = g->f64.ssrc;
    ba.fac = g->f64.fac;
    ba.ofac = g->f64.ofac;
    ba.eta = eta[i];
    ba.khu = g->f32.khu;
    ba.khv = g->f32.khv;
    ba.pb = g->f32.pb;
    ba.sp7 = g->f32.sp7;
    ba.eu = g->f32.un;
    ba.ev = g->f32.vn;
    ba.bc4 = g->bc_order == 4 ? 1 : 0;
    ba.zfac = g->f64.zfac;
    hba[i] = ba;
    hrb[i] = RebaseArgs{g->f64.un, g->f64.vn, g->f32.un, g->f32.vn, (int)g->G};
    if (reps) {
      reps[i].steps_taken = 0;
      reps[i].fp32_steps = 0;
      reps[i].residual = NAN;
      reps[i].dt_used = dt;
      reps[i].n_history = 0;
      reps[i].resident_fallbacks = 0;
    }
  }
  HR_HIPB(hipMemcpyAsync(b->sa64, h64.data(), h64.size() * sizeof(h64[0]), hipMemcpyHostToDevice, b->stream));
  HR_HIPB(hipMemcpyAsync(b->sa32, h32.data(), h32.size() * sizeof(h32[0]), hipMemcpyHostToDevice, b->stream));
  HR_HIPB(hipMemcpyAsync(b->ra, hra.data(), hra.size() * sizeof(hra[0]), hipMemcpyHostToDevice, b->stream));
  HR_HIPB(hipMemcpyAsync(b->ba, hba.data(), hba.size() * sizeof(hba[0]), hipMemcpyHostToDevice, b->stream));
  HR_HIPB(hipMemcpyAsync(b->rb, hrb.data(), hrb.size() * sizeof(hrb[0]), hipMemcpyHostToDevice, b->stream));
  HR_HIPB(launch_fill(reinterpret_cast<float*>(b->rerr), 0.0f, 1, b->stream));
  HR_HIPB(hipStreamSynchronize(b->stream));

  const long max_cycles = (n_steps + K - 1) / K;
  bool lists_dirty = true;
  int mode = 0;
  for (long cyc = 0; cyc < max_cycles; ++cyc) {
    if (lists_dirty) {
      hr_status st = upload_lists(b, run, K, &mode);
      if (st != HR_OK) return st;
      lists_dirty = false;
    }
    if (mode == 0) break;
    if (!b->exec || b->exec_mode != mode || b->exec_K != K || b->exec_sig != b->groups_sig) {
      hr_status st = capture(b, mode, K);
      if (st != HR_OK) return st;
    }
    HR_HIPB(hipGraphLaunch(b->exec, b->stream));
    HR_HIPB(hipMemcpyAsync(b->host_out, b->out, b->n * sizeof(double), hipMemcpyDeviceToHost,
                           b->stream));
    unsigned* err_word = reinterpret_cast<unsigned*>(b->host_out + b->n);
    if (!b->groups.empty())
      HR_HIPB(hipMemcpyAsync(err_word, b->rerr, sizeof(unsigned), hipMemcpyDeviceToHost,
                             b->stream));
    HR_HIPB(hipStreamSynchronize(b->stream));
    if (!b->groups.empty() && *err_word) {
      *err_word = 0;
      return bfail(HR_EDEVICE, "resident kernel in a batch: an exchange wait timed out");
    }
    for (int i = 0; i < b->n; ++i) {
      GridRun& r = run[i];
      if (r.done) continue;
      r.steps += K;
      if (r.phase == 0) r.f32steps += K;
      const double res = b->host_out[i];
      r.last = res;
      if (reps) {
        hr_relax_report& rp = reps[i];
        if (rp.history && rp.n_history < rp.history_cap) rp.history[rp.n_history] = res;
        rp.n_history++;
      }
      if (!std::isfinite(res)) {
        r.done = true;
        r.why = 2;
        lists_dirty = true;
        continue;
      }
      if (tol > 0 && res < tol) {
        r.done = true;
        r.why = 1;
        lists_dirty = true;
        continue;
      }
      if (r.phase == 0) {
        if (res < r.best) {
          r.best = res;
          r.stall = 0;
        } else {
          ++r.stall;
        }
        const hr_grid* g = b->g[i];
        if (res < r.sw || r.stall >= g->sw_stall ||
            (g->sw_max_steps > 0 && r.steps >= g->sw_max_steps)) {
          r.phase = 1;
          lists_dirty = true;
        }
      }
    }
  }
  HR_HIPB(hipStreamSynchronize(b->stream));
  bool nonfinite = false, notconv = false;
  for (int i = 0; i < b->n; ++i) {
    if (reps) {
      reps[i].steps_taken = run[i].steps;
      reps[i].fp32_steps = run[i].f32steps;
      reps[i].residual = run[i].last;
    }
    if (run[i].why == 2) nonfinite = true;
    if (tol > 0 && run[i].why != 1) notconv = true;
  }
  if (nonfinite) return bfail(HR_ENONFINITE, "a batched grid's residual is not finite");
  if (notconv) return bfail(HR_ENOTCONV, "a batched grid did not reach the tolerance");
  return HR_OK;
}

}  // extern "C"
