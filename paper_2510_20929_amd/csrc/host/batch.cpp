// Batched uneven reconstructions: many independent datasets in one persistent launch
// per frame-size class, captured once into a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../../include/ptyhip.h"
#include "../kernels/launch.hpp"
#include "plan.hpp"

using namespace ptyhip;

namespace {

struct Bound {
  const float *obj = nullptr, *probe = nullptr, *weights = nullptr, *pos = nullptr, *imeas = nullptr;
  double* loss = nullptr;
  float *g_obj = nullptr, *g_probe = nullptr, *g_pos = nullptr, *g_w = nullptr;
  bool set = false;
};

}  // namespace

struct ptyhip_batch_s {
  int n = 0;
  int device = 0;
  int cls_first[BATCH_CLASSES] = {};  // table entries of each class (sorted table)
  int cls_count[BATCH_CLASSES] = {};
  int cls_wg[BATCH_CLASSES] = {};     // workgroups of each class's launch
  std::vector<Plan*> plans;
  std::vector<int> K, first_wg, n_wg;
  std::vector<Bound> bound;
  std::vector<BatchEntry> tab;
  BatchEntry* staging = nullptr;  // pinned copy of the table, source of the upload
  BatchEntry* dev_tab = nullptr;
  bool uploaded = false;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;  // capture stream (capture is not allowed on the legacy default stream)
  uint32_t graph_flags = 0xffffffffu;
  // concurrent classes: each class's launch and follow-up reductions on a branch of its own,
  // the classes sharing the CUs in proportion to their work
  bool concurrent = false;
  hipStream_t side[BATCH_CLASSES] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[BATCH_CLASSES] = {};
  ~ptyhip_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipStream_t s : side)
      if (s) (void)hipStreamDestroy(s);
    if (fork) (void)hipEventDestroy(fork);
    for (hipEvent_t e : join)
      if (e) (void)hipEventDestroy(e);
    if (cap) (void)hipStreamDestroy(cap);
    if (graph) (void)hipGraphDestroy(graph);
    if (dev_tab) (void)hipFree(dev_tab);
    if (staging) (void)hipHostFree(staging);
    for (Plan* p : plans) delete p;
  }
};

extern "C" {

ptyhip_status ptyhip_batch_create(const ptyhip_desc* descs, const int32_t* K, int32_t n, const ptyhip_tune* tune,
                                  ptyhip_batch* out) {
  if (!out) return PTYHIP_EINVAL;
  *out = nullptr;
  if (!descs || !K || n < 1 || n > 1024) return PTYHIP_EINVAL;
  if (tune && (tune->variant < 0 || tune->variant > 1 || tune->grid < 0)) return PTYHIP_EINVAL;
  for (int i = 0; i < n; ++i) {
    ptyhip_status s = validate_desc(&descs[i]);
    if (s != PTYHIP_OK) return s;
    const int N = descs[i].frame;
    if (N < 64 || descs[i].n_slices != 1 || descs[i].propagation != PTYHIP_PROP_FAR ||
        descs[i].subpixel != PTYHIP_SUBPIXEL_BILINEAR)
      return PTYHIP_EUNSUPPORTED;
    if (K[i] < 0) return PTYHIP_EBOUNDS;
  }
  auto* b = new (std::nothrow) ptyhip_batch_s();
  if (!b) return PTYHIP_ENOMEM;
  b->n = n;
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return PTYHIP_EHIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
    delete b;
    return PTYHIP_EHIP;
  }
  // work of each dataset: positions x modes x (N^2 log2 N^2) transform cost
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) {
    const double N = descs[i].frame;
    cost[i] = double(std::max(K[i], 1)) * descs[i].n_modes * N * N * std::log2(N * N);
  }
  // per frame-size class: one workgroup per CU (a tuned total if given), one workgroup per
  // dataset at least, the rest by largest remainder in proportion to the work; inside a
  // class the most expensive datasets take the first workgroups. Concurrent classes
  // (tune variant 1) split that total among the classes in proportion to their work.
  b->concurrent = tune && tune->variant == 1;
  b->n_wg.assign(n, 1);
  b->first_wg.assign(n, 0);
  const int grid_total = (tune && tune->grid > 0) ? int(tune->grid) : prop.multiProcessorCount;
  double cls_cost[BATCH_CLASSES] = {}, all_cost = 0.0;
  for (int i = 0; i < n; ++i) {
    cls_cost[batch_class(descs[i].frame, descs[i].loss)] += cost[i];
    all_cost += cost[i];
  }
  for (int c = 0; c < BATCH_CLASSES; ++c) {
    std::vector<int> members;
    for (int i = 0; i < n; ++i)
      if (batch_class(descs[i].frame, descs[i].loss) == c) members.push_back(i);
    const int nc = int(members.size());
    b->cls_count[c] = nc;
    if (nc == 0) continue;
    const int share = b->concurrent ? int(std::lround(double(grid_total) * cls_cost[c] / all_cost)) : grid_total;
    const int total = std::max(nc, share);
    b->cls_wg[c] = total;
    double tot = 0.0;
    for (int i : members) tot += cost[i];
    const int left = total - nc;
    std::vector<double> rem(n, 0.0);
    int given = 0;
    for (int i : members) {
      const double share = cost[i] / tot * left;
      const int w = int(std::floor(share));
      b->n_wg[i] += w;
      given += w;
      rem[i] = share - w;
    }
    std::vector<int> order = members;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return rem[x] > rem[y]; });
    for (int j = 0; j < left - given; ++j) b->n_wg[order[j % nc]] += 1;
    std::sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    int w0 = 0;
    for (int i : order) {
      b->first_wg[i] = w0;
      w0 += b->n_wg[i];
    }
  }
  b->cls_first[0] = 0;
  for (int c = 1; c < BATCH_CLASSES; ++c) b->cls_first[c] = b->cls_first[c - 1] + b->cls_count[c - 1];
  b->K.assign(K, K + n);
  b->bound.resize(n);
  b->plans.assign(n, nullptr);
  for (int i = 0; i < n; ++i) {
    Plan* p = new (std::nothrow) Plan();
    if (!p) {
      delete b;
      return PTYHIP_ENOMEM;
    }
    b->plans[i] = p;
    ptyhip_tune t{};
    if (tune) t = *tune;
    t.mode_groups = 0;  // a batch runs whole positions per workgroup
    t.grid = std::max(b->n_wg[i], prop.multiProcessorCount);
    // the body each class's launch runs: 128^2 the register-resident patch layout with
    // recomputed far fields (several modes), the others the default layout
    t.variant = batch_variant(descs[i].frame);
    t.recompute = (descs[i].frame == 128 && descs[i].n_modes > 1) ? 1 : 0;
    if (t.plain_chunk <= 0) t.plain_chunk = 128;
    p->whole_windows = true;
    ptyhip_status s = plan_init(p, descs[i], std::max(K[i], 1), &t);
    if (s != PTYHIP_OK) {
      delete b;
      return s;
    }
    // the batched launch runs the same bodies: its scratch layout must be the plan's
    size_t off = 0;
    const size_t need = batched_scratch_elems(descs[i].frame, descs[i].n_modes, descs[i].n_eig, t.recompute, &off);
    if (need > p->scratch_stride || off != p->pacc_off) {
      delete b;
      return PTYHIP_EUNSUPPORTED;
    }
  }
  b->tab.resize(n);
  if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return PTYHIP_EHIP;
  }
  if (b->concurrent) {
    bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess;
    for (int c = 0; c < BATCH_CLASSES && ok; ++c)
      ok = hipStreamCreateWithFlags(&b->side[c], hipStreamNonBlocking) == hipSuccess &&
           hipEventCreateWithFlags(&b->join[c], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
      delete b;
      return PTYHIP_EHIP;
    }
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&b->staging), sizeof(BatchEntry) * n, hipHostMallocDefault) !=
          hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&b->dev_tab), sizeof(BatchEntry) * n) != hipSuccess) {
    delete b;
    return PTYHIP_ENOMEM;
  }
  *out = reinterpret_cast<ptyhip_batch>(b);
  return PTYHIP_OK;
}

ptyhip_status ptyhip_batch_bind(ptyhip_batch bh, int32_t i, const float* obj, const float* probe,
                                const float* weights, const float* positions, const float* I_meas, double* loss,
                                float* g_obj, float* g_probe, float* g_pos, float* g_weights) {
  auto* b = reinterpret_cast<ptyhip_batch_s*>(bh);
  if (!b || i < 0 || i >= b->n) return PTYHIP_EINVAL;
  if (!obj || !probe || !loss || (b->K[i] > 0 && (!positions || !I_meas))) return PTYHIP_EINVAL;
  if (b->plans[i]->d.n_eig > 1 && b->K[i] > 0 && !weights) return PTYHIP_EINVAL;
  Bound& d = b->bound[i];
  d.obj = obj;
  d.probe = probe;
  d.weights = weights;
  d.pos = positions;
  d.imeas = I_meas;
  d.loss = loss;
  d.g_obj = g_obj;
  d.g_probe = g_probe;
  d.g_pos = g_pos;
  d.g_w = g_weights;
  d.set = true;
  return PTYHIP_OK;
}

ptyhip_status ptyhip_batch_launch(ptyhip_batch bh, void* stream, uint32_t flags) {
  auto* b = reinterpret_cast<ptyhip_batch_s*>(bh);
  if (!b) return PTYHIP_EINVAL;
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (hipSetDevice(b->device) != hipSuccess) return PTYHIP_EHIP;
  const uint32_t grads = flags & (PTYHIP_GRAD_OBJ | PTYHIP_GRAD_PROBE | PTYHIP_GRAD_POS | PTYHIP_GRAD_WEIGHTS);
  for (int i = 0; i < b->n; ++i) {
    const Bound& d = b->bound[i];
    if (!d.set) return PTYHIP_EINVAL;
    if (((grads & PTYHIP_GRAD_OBJ) && !d.g_obj) || ((grads & PTYHIP_GRAD_PROBE) && !d.g_probe) ||
        ((grads & PTYHIP_GRAD_POS) && b->K[i] > 0 && !d.g_pos) ||
        ((grads & PTYHIP_GRAD_WEIGHTS) && b->K[i] > 0 && (!d.g_w || !d.weights)))
      return PTYHIP_EINVAL;
  }
  if (flags & (PTYHIP_PLAIN | PTYHIP_BATCH_PER_CALL)) {
    const uint32_t f = grads | (flags & PTYHIP_PLAIN);
    for (int i = 0; i < b->n; ++i) {
      const Bound& d = b->bound[i];
      ptyhip_status s = call_forward_adjoint(b->plans[i], st, b->K[i], f, d.obj, d.probe, d.weights, d.pos, d.imeas,
                                             d.loss, nullptr, d.g_obj, d.g_probe, d.g_pos, d.g_w, nullptr, false);
      if (s != PTYHIP_OK) return s;
    }
    return PTYHIP_OK;
  }
  // descriptor table for these flags
  for (int i = 0; i < b->n; ++i) {
    const Bound& d = b->bound[i];
    Plan* p = b->plans[i];
    const bool wo = grads & PTYHIP_GRAD_OBJ, wp = grads & PTYHIP_GRAD_PROBE, wq = grads & PTYHIP_GRAD_POS,
               ww = grads & PTYHIP_GRAD_WEIGHTS;
    BatchEntry e;
    std::memset(&e, 0, sizeof(e));
    e.a = make_args(p, b->K[i], grads ? MODE_FWD_ADJ : MODE_FORWARD, true, d.obj, d.probe, d.weights, d.pos, d.imeas,
                    nullptr, nullptr, nullptr, wo ? d.g_obj : nullptr, wp, wq, ww);
    e.a.zero_acc = 1;
    if (wo) {
      e.g.gwin = p->gwin;
      e.g.wvalid = p->wvalid;
      e.g.pos = d.pos;
      e.g.gobj = reinterpret_cast<float2*>(d.g_obj);
      e.g.K = b->K[i];
      e.g.S = p->d.n_slices;
      e.g.N = p->d.frame;
      e.g.H = p->d.obj_h;
      e.g.W = p->d.obj_w;
      e.g.accumulate = 0;
    }
    e.g_probe = wp ? reinterpret_cast<float2*>(d.g_probe) : nullptr;
    e.loss = d.loss;
    e.g_pos = wq ? d.g_pos : nullptr;
    e.g_w = ww ? d.g_w : nullptr;
    e.first_wg = b->first_wg[i];
    e.n_wg = b->n_wg[i];
    e.N = p->d.frame;
    b->tab[i] = e;
  }
  // each class's kernel finds a workgroup's dataset by first_wg among the class's
  // entries, so upload by class, then in first_wg order
  std::vector<int> order(b->n);
  std::iota(order.begin(), order.end(), 0);
  std::sort(order.begin(), order.end(), [&](int x, int y) {
    const int cx = batch_class(b->tab[x].N, b->tab[x].a.loss), cy = batch_class(b->tab[y].N, b->tab[y].a.loss);
    return cx != cy ? cx < cy : b->first_wg[x] < b->first_wg[y];
  });
  std::vector<BatchEntry> sorted(b->n);
  for (int j = 0; j < b->n; ++j) sorted[j] = b->tab[order[j]];
  // the gather launch of a class: each dataset with an object gradient owns a range of
  // its workgroups, one per tile
  for (int j = 0, tile = 0; j < b->n; ++j) {
    BatchEntry& e = sorted[j];
    if (j > 0 && batch_class(e.N, e.a.loss) != batch_class(sorted[j - 1].N, sorted[j - 1].a.loss)) tile = 0;
    e.first_tile = tile;
    if (e.g.gobj) {
      e.gts = gather_tile_side(e.g.H, e.g.W, e.g.S);
      e.tiles_x = (e.g.W + e.gts - 1) / e.gts;
      e.tiles_y = (e.g.H + e.gts - 1) / e.gts;
      tile += e.tiles_x * e.tiles_y * e.g.S;
    }
  }
  if (!b->uploaded || std::memcmp(sorted.data(), b->staging, sizeof(BatchEntry) * b->n) != 0) {
    // the previous upload may still be in flight or in use: wait for the stream first
    if (hipStreamSynchronize(st) != hipSuccess) return PTYHIP_EHIP;
    std::memcpy(b->staging, sorted.data(), sizeof(BatchEntry) * b->n);
    if (hipMemcpyAsync(b->dev_tab, b->staging, sizeof(BatchEntry) * b->n, hipMemcpyHostToDevice, st) != hipSuccess)
      return PTYHIP_EHIP;
    b->uploaded = true;
  }
  if (!b->exec || b->graph_flags != grads) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    // capture records the launches without running them; the graph then runs on `st`
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return PTYHIP_EHIP;
    hipError_t e = hipSuccess;
    if (b->concurrent) {
      // fork: every class's branch waits for the capture stream, then runs on its own stream;
      // join: the capture stream waits for every branch
      e = hipEventRecord(b->fork, b->cap);
      for (int c = 0; c < BATCH_CLASSES && e == hipSuccess; ++c) {
        if (b->cls_count[c] == 0) continue;
        e = hipStreamWaitEvent(b->side[c], b->fork, 0);
        if (e == hipSuccess)
          e = launch_batched_class(b->dev_tab, sorted.data(), c, b->cls_first, b->cls_count, b->cls_wg, b->side[c]);
        if (e == hipSuccess) e = hipEventRecord(b->join[c], b->side[c]);
        if (e == hipSuccess) e = hipStreamWaitEvent(b->cap, b->join[c], 0);
      }
    } else {
      e = launch_batched(b->dev_tab, sorted.data(), b->n, b->cls_first, b->cls_count, b->cls_wg, b->cap);
    }
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess || !g) return PTYHIP_EHIP;
    b->graph = g;
    if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) return PTYHIP_EHIP;
    b->graph_flags = grads;
  }
  return hipGraphLaunch(b->exec, st) == hipSuccess ? PTYHIP_OK : PTYHIP_EHIP;
}

ptyhip_status ptyhip_batch_get_error(ptyhip_batch bh, void* stream, uint32_t* flags) {
  auto* b = reinterpret_cast<ptyhip_batch_s*>(bh);
  if (!b || !flags) return PTYHIP_EINVAL;
  uint32_t f = 0;
  for (Plan* p : b->plans) {
    uint32_t g = 0;
    ptyhip_status s = ptyhip_get_error(reinterpret_cast<ptyhip_plan>(p), stream, &g);
    if (s != PTYHIP_OK) return s;
    f |= g;
  }
  *flags = f;
  return PTYHIP_OK;
}

void ptyhip_batch_destroy(ptyhip_batch bh) {
  auto* b = reinterpret_cast<ptyhip_batch_s*>(bh);
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  delete b;
}

}  // extern "C"
