// Batched solves: many independent problems (uneven shapes, vector
// right-hand sides) run as ONE hipGraph launch of grouped pass kernels.
//
// For each pass, the problems that use the same compiled kernel form
// grouped launches (the kernel finds its problem from a block -> entry map);
// a group whose algorithmic bytes exceed a quarter of the pass's is split
// into several launches.  The launches of a pass are dealt, longest first
// by bytes, to the least loaded of kChains chains; the chains are parallel
// branches of the graph, each a sequence of launches, and the five passes
// are joined in order.  (Left to the runtime, ten or more branches per pass
// are spread over the process's hardware queues in capture order, and the
// two longest launches of a pass can land on the same queue, one after the
// other, while the others idle.)  The caller's f and u pointers are written
// to a small device table by one kernel per call, so the graph itself never
// changes between solves.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/ups.h"
#include "green.hpp"
#include "passes.hpp"
#include "plan.hpp"
#include "trace.hpp"

using namespace ups;

namespace {

constexpr int kMaxBatch = 200;
// parallel chains per pass: the hardware queues a process gets by default
constexpr int kChains = 4;

struct IoPtrs {
  const void* p[2 * kMaxBatch];
};

__global__ void k_set_io(IoPtrs ptrs, int n, const void** dst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = ptrs.p[i];
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Launch {
  const PassVariant* var;
  double bytes = 0;              // algorithmic bytes of its problems in this pass
  std::vector<int> probs;        // problem indices in this group
  size_t off_ents = 0, off_bmap = 0;
  unsigned nblocks = 0;
  std::vector<GroupEntry> ents;  // host copy (pointers filled at setup)
  std::vector<unsigned short> bmap;
};

}  // namespace

struct ups_batch_s {
  std::vector<ups_problem> probs;
  std::vector<PlanGeom> geo;
  std::vector<std::array<const PassVariant*, 5>> var;
  std::vector<size_t> off_green, off_work;
  std::vector<Launch> launches[5];
  std::vector<int> chains[5][kChains];   // launch indices of each chain, in order
  size_t off_tables = 0, off_io = 0;
  size_t green_bytes = 0, work_bytes = 0;
  void* green = nullptr;
  void* work = nullptr;
  bool ready = false;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> events;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;

  ~ups_batch_s() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    for (hipEvent_t e : events) hipEventDestroy(e);
    for (hipStream_t s : streams) hipStreamDestroy(s);
  }
};

namespace ups {
const PassVariant* tuned_variant(PassKind kind, bool f64, int length, const PlanGeom& g);
}

static const PassKind kKinds[5] = {PASS_XFWD, PASS_YFWD, PASS_ZCONV, PASS_YINV, PASS_XINV};

extern "C" {

ups_status ups_batch_create(const ups_problem* probs, int count, ups_batch_t* out) {
  if (!out) return set_error(UPS_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!probs || count < 1) return set_error(UPS_ERR_INVALID_ARG, "need at least one problem");
  if (count > kMaxBatch) return set_error(UPS_ERR_UNSUPPORTED, "a batch holds at most 200 problems");
  ups_batch_s* b = new ups_batch_s();
  size_t green_off = 0, work_off = 0, setup_max = 0;
  for (int i = 0; i < count; ++i) {
    PlanGeom g{};
    ups_status s = validate_problem(&probs[i], &g);
    if (s != UPS_OK) {
      delete b;
      return s;
    }
    plan_layout(g);
    std::array<const PassVariant*, 5> v{};
    const int len[5] = {g.mx, g.my, g.mz, g.my, g.mx};
    for (int k = 0; k < 5; ++k) {
      v[k] = tuned_variant(kKinds[k], g.f64, len[k], g);
      if (!v[k]) {
        delete b;
        return set_error(UPS_ERR_UNSUPPORTED, "no kernel for a pass of a batch problem");
      }
    }
    b->probs.push_back(probs[i]);
    b->geo.push_back(g);
    b->var.push_back(v);
    b->off_green.push_back(green_off);
    green_off = align_up(green_off + g.green_bytes, 256);
    b->off_work.push_back(work_off);
    work_off = align_up(work_off + g.solve_work, 256);
    setup_max = std::max(setup_max, g.work_bytes);
  }
  // group problems per pass by kernel variant, split groups above a quarter
  // of the pass's bytes, and deal the launches to the chains longest first
  for (int k = 0; k < 5; ++k) {
    std::map<const PassVariant*, std::vector<int>> groups;
    double total = 0;
    for (int i = 0; i < count; ++i) {
      groups[b->var[i][k]].push_back(i);
      total += model_bytes(b->geo[i], k);
    }
    const double cap = total / kChains;
    for (auto& kv : groups) {
      std::vector<int>& ps = kv.second;
      std::stable_sort(ps.begin(), ps.end(), [&](int a, int c) {
        return model_bytes(b->geo[a], k) > model_bytes(b->geo[c], k);
      });
      // first fit, largest problem first, into launches of at most `cap`
      // bytes (a larger problem gets a launch of its own)
      std::vector<Launch> pieces;
      for (int i : ps) {
        const double c = model_bytes(b->geo[i], k);
        Launch* dst = nullptr;
        for (Launch& L : pieces)
          if (L.bytes + c <= cap) {
            dst = &L;
            break;
          }
        if (!dst) {
          pieces.emplace_back();
          dst = &pieces.back();
          dst->var = kv.first;
        }
        dst->probs.push_back(i);
        dst->bytes += c;
      }
      for (Launch& L : pieces) b->launches[k].push_back(std::move(L));
    }
    std::vector<int> order(b->launches[k].size());
    for (size_t j = 0; j < order.size(); ++j) order[j] = int(j);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int c) { return b->launches[k][a].bytes > b->launches[k][c].bytes; });
    double load[kChains] = {};
    for (int j : order) {
      int best = 0;
      for (int c = 1; c < kChains; ++c)
        if (load[c] < load[best]) best = c;
      b->chains[k][best].push_back(j);
      load[best] += b->launches[k][j].bytes;
    }
    for (Launch& L : b->launches[k]) {
      unsigned block = 0;
      for (int e = 0; e < int(L.probs.size()); ++e) {
        const int i = L.probs[e];
        PassArgs a = make_args(b->geo[i], nullptr);
        int gx, gy, gz;
        const unsigned nb = unsigned(blocks_for(*L.var, a, &gx, &gy, &gz));
        GroupEntry ent{};
        ent.block0 = block;
        ent.nblocks = nb;
        ent.io_in = ent.io_out = -1;
        L.ents.push_back(ent);
        L.bmap.insert(L.bmap.end(), nb, (unsigned short)e);
        block += nb;
        const unsigned pad = (8 - block % 8) % 8;   // keep every block0 a multiple of 8
        L.bmap.insert(L.bmap.end(), pad, (unsigned short)e);
        block += pad;
      }
      L.nblocks = block;
    }
  }
  // device tables after the per-problem green regions
  size_t off = green_off;
  b->off_tables = off;
  for (int k = 0; k < 5; ++k)
    for (Launch& L : b->launches[k]) {
      L.off_ents = off;
      off = align_up(off + sizeof(GroupEntry) * L.ents.size(), 256);
      L.off_bmap = off;
      off = align_up(off + sizeof(unsigned short) * L.bmap.size(), 256);
    }
  b->off_io = off;
  off = align_up(off + sizeof(void*) * 2 * count, 256);
  b->green_bytes = off;
  b->work_bytes = std::max(work_off, setup_max);
  if (log_level() >= 2) {
    logf(2, "batch %p: %d problems; grouped launches per pass %zu %zu %zu %zu %zu; G_hat buffer %zu B, work %zu B",
         static_cast<void*>(b), count, b->launches[0].size(), b->launches[1].size(), b->launches[2].size(),
         b->launches[3].size(), b->launches[4].size(), b->green_bytes, b->work_bytes);
    for (int k = 0; k < 5; ++k)
      for (const Launch& L : b->launches[k])
        logf(2, "batch %p pass %d: %s, %zu problem(s), %u blocks, %.0f model bytes", static_cast<void*>(b), k,
             L.var->name, L.probs.size(), L.nblocks, L.bytes);
  }
  *out = b;
  set_error(UPS_OK, "");
  return UPS_OK;
}

ups_status ups_batch_sizes(ups_batch_t b, size_t* green_bytes, size_t* work_bytes) {
  if (!b) return set_error(UPS_ERR_INVALID_ARG, "batch is NULL");
  if (green_bytes) *green_bytes = b->green_bytes;
  if (work_bytes) *work_bytes = b->work_bytes;
  set_error(UPS_OK, "");
  return UPS_OK;
}

ups_status ups_batch_setup(ups_batch_t b, void* green, size_t green_bytes, void* work, size_t work_bytes,
                           void* stream) {
  if (!b) return set_error(UPS_ERR_INVALID_ARG, "batch is NULL");
  if (!green || !work) return set_error(UPS_ERR_INVALID_ARG, "green and work must be device pointers");
  if ((reinterpret_cast<uintptr_t>(green) | reinterpret_cast<uintptr_t>(work)) & 255)
    return set_error(UPS_ERR_INVALID_ARG, "green and work must be 256-byte aligned");
  if (green_bytes < b->green_bytes || work_bytes < b->work_bytes)
    return set_error(UPS_ERR_WORKSPACE, "batch buffers smaller than ups_batch_sizes");
  if (b->ready) return set_error(UPS_ERR_STATE, "ups_batch_setup already ran on this batch");
  int dev = 0;
  ups_status s = check_device(&dev);
  if (s != UPS_OK) return s;
  hipStream_t st = static_cast<hipStream_t>(stream);
  char* gb = static_cast<char*>(green);
  char* wb = static_cast<char*>(work);
  const int n = int(b->probs.size());
  hipError_t e = hipSuccess;
  // G_hat and twiddles of every problem (the whole work buffer is scratch here)
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const PlanGeom& g = b->geo[i];
    char* pg = gb + b->off_green[i];
    e = build_twiddles(g.f64, g.mx, pg + g.off_twx, wb, st);
    if (e == hipSuccess) e = build_twiddles(g.f64, g.my, pg + g.off_twy, wb, st);
    if (e == hipSuccess) e = build_twiddles(g.f64, g.mz, pg + g.off_twz, wb, st);
    if (e == hipSuccess) e = build_green(g.f64, g.bc, g.green, g.oz, g.oy, g.kx, g.gz, g.h, g.mx, g.my, g.mz, pg + g.off_ghat, wb, st);
  }
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  // descriptor tables
  const void* const* io = reinterpret_cast<const void* const*>(gb + b->off_io);
  for (int k = 0; k < 5; ++k) {
    for (Launch& L : b->launches[k]) {
      for (int j = 0; j < int(L.probs.size()); ++j) {
        const int i = L.probs[j];
        GroupEntry& ent = L.ents[j];
        ent.a = make_args(b->geo[i], gb + b->off_green[i]);
        void* W = wb + b->off_work[i];
        ent.in = W;
        ent.out = W;
        if (k == 0) ent.io_in = 2 * i;
        if (k == 4) ent.io_out = 2 * i + 1;
      }
      e = hipMemcpy(gb + L.off_ents, L.ents.data(), sizeof(GroupEntry) * L.ents.size(), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(gb + L.off_bmap, L.bmap.data(), sizeof(unsigned short) * L.bmap.size(),
                      hipMemcpyHostToDevice);
      if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
    }
  }
  // the graph: five joined stages, one branch per chain of grouped launches
  for (int i = 0; i < kChains + 1 && e == hipSuccess; ++i) {
    hipStream_t s2;
    e = hipStreamCreateWithFlags(&s2, hipStreamNonBlocking);
    if (e == hipSuccess) b->streams.push_back(s2);
  }
  for (int i = 0; i < 5 * (kChains + 1) && e == hipSuccess; ++i) {
    hipEvent_t ev;
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) b->events.push_back(ev);
  }
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  hipStream_t cap = b->streams[0];
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  size_t ev_i = 0;
  for (int k = 0; k < 5 && e == hipSuccess; ++k) {
    hipEvent_t fork = b->events[ev_i++];
    e = hipEventRecord(fork, cap);
    for (int c = 0; c < kChains && e == hipSuccess; ++c) {
      if (b->chains[k][c].empty()) continue;
      hipStream_t sc = b->streams[1 + c];
      e = hipStreamWaitEvent(sc, fork, 0);
      for (size_t q = 0; q < b->chains[k][c].size() && e == hipSuccess; ++q) {
        Launch& L = b->launches[k][b->chains[k][c][q]];
        GroupArgs ga{reinterpret_cast<const GroupEntry*>(gb + L.off_ents),
                     reinterpret_cast<const unsigned short*>(gb + L.off_bmap), io};
        L.var->launch_grouped(ga, L.nblocks, sc);
        e = hipGetLastError();
      }
      hipEvent_t join = b->events[ev_i++];
      if (e == hipSuccess) e = hipEventRecord(join, sc);
      if (e == hipSuccess) e = hipStreamWaitEvent(cap, join, 0);
    }
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = hipStreamEndCapture(cap, &graph);
  if (e == hipSuccess) e = e2;
  if (e == hipSuccess) e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
  b->graph = graph;
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  e = hipStreamSynchronize(st);
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  b->green = green;
  b->work = work;
  b->ready = true;
  set_error(UPS_OK, "");
  return UPS_OK;
}

ups_status ups_batch_solve(ups_batch_t b, const void* const* f, void* const* u, void* stream) {
  if (!b) return set_error(UPS_ERR_INVALID_ARG, "batch is NULL");
  if (!b->ready) return set_error(UPS_ERR_STATE, "ups_batch_setup has not completed on this batch");
  if (!f || !u) return set_error(UPS_ERR_INVALID_ARG, "f and u must be arrays of device pointers");
  const int n = int(b->probs.size());
  IoPtrs ptrs{};
  for (int i = 0; i < n; ++i) {
    const uintptr_t al = 2 * b->geo[i].elem - 1;
    if (!f[i] || !u[i]) return set_error(UPS_ERR_INVALID_ARG, "null array in the batch");
    if ((reinterpret_cast<uintptr_t>(f[i]) | reinterpret_cast<uintptr_t>(u[i])) & al)
      return set_error(UPS_ERR_INVALID_ARG, "misaligned array in the batch");
    ptrs.p[2 * i] = f[i];
    ptrs.p[2 * i + 1] = u[i];
  }
  TraceRange range("ups_batch_solve");
  logf(3, "batch solve %p: %d problems, stream %p", static_cast<void*>(b), n, stream);
  hipStream_t st = static_cast<hipStream_t>(stream);
  const void** io = reinterpret_cast<const void**>(static_cast<char*>(b->green) + b->off_io);
  hipLaunchKernelGGL(k_set_io, dim3((2 * n + 255) / 256), dim3(256), 0, st, ptrs, 2 * n, io);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipGraphLaunch(b->exec, st);
  if (e != hipSuccess) return set_error(UPS_ERR_DEVICE, hipGetErrorString(e));
  set_error(UPS_OK, "");
  return UPS_OK;
}

int ups_batch_launches(ups_batch_t b, int pass) {
  if (!b || pass < 0 || pass > 4) return 0;
  return int(b->launches[pass].size());
}

ups_status ups_batch_destroy(ups_batch_t b) {
  delete b;
  set_error(UPS_OK, "");
  return UPS_OK;
}

}  // extern "C"
