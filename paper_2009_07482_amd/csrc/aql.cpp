// AQL queue dispatch; see aql.hpp.
#include "aql.hpp"

#include <dlfcn.h>
#include <hip/hip_runtime.h>
#include <hsa/hsa.h>
#include <hsa/hsa_ext_amd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <thread>

#if defined(__x86_64__)
#include <immintrin.h>
#define PSC_AQL_PAUSE() _mm_pause()
#else
#define PSC_AQL_PAUSE() ((void)0)
#endif

namespace psc {

namespace {

#define PSC_HSA(call)                                                                        \
  do {                                                                                       \
    hsa_status_t s_ = (call);                                                                \
    if (s_ != HSA_STATUS_SUCCESS) fail(PSC_ERR_HIP, std::string(#call) + ": " + hsa_msg(s_)); \
  } while (0)

#define PSC_HIPA(call)                                                                            \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) fail(PSC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

std::string hsa_msg(hsa_status_t s) {
  const char *m = nullptr;
  if (hsa_status_string(s, &m) == HSA_STATUS_SUCCESS && m) return m;
  return "HSA status " + std::to_string(int(s));
}

// Implicit argument kinds the host fills (codes of libpsc_kernels.kargs).
enum Hidden : int {
  kHidUnknown = 0, kBlockCountX = 1, kBlockCountY, kBlockCountZ, kGroupSizeX, kGroupSizeY, kGroupSizeZ,
  kRemainderX, kRemainderY, kRemainderZ, kGlobalOffsetX, kGlobalOffsetY, kGlobalOffsetZ, kGridDims
};

struct KernelMeta {
  uint32_t explicit_bytes = 0;
  std::vector<std::pair<uint32_t, int>> hidden;  // (offset, kind)
};

// The library's code object and its argument table, found beside libpsc.so.
struct CodeObject {
  std::string dir;
  std::vector<char> bytes;
  std::map<std::string, KernelMeta> meta;
  std::string error;
};

const CodeObject &code_object() {
  static CodeObject co = [] {
    CodeObject c;
    Dl_info info{};
    if (!dladdr(reinterpret_cast<const void *>(&code_object), &info) || !info.dli_fname) {
      c.error = "cannot locate the library file";
      return c;
    }
    std::string lib = info.dli_fname;
    c.dir = lib.substr(0, lib.find_last_of('/') + 1);
    std::ifstream f(c.dir + "libpsc_kernels.hsaco", std::ios::binary);
    if (!f) {
      c.error = c.dir + "libpsc_kernels.hsaco is missing (built with libpsc.so)";
      return c;
    }
    c.bytes.assign(std::istreambuf_iterator<char>(f), std::istreambuf_iterator<char>());
    std::ifstream m(c.dir + "libpsc_kernels.kargs");
    if (!m) {
      c.error = c.dir + "libpsc_kernels.kargs is missing (built with libpsc.so)";
      return c;
    }
    // one kernel per line: name explicit_bytes n_hidden offset:kind ...
    std::string line;
    while (std::getline(m, line)) {
      std::istringstream ls(line);
      std::string name;
      KernelMeta km;
      int n = 0;
      if (!(ls >> name >> km.explicit_bytes >> n)) continue;
      for (int i = 0; i < n; ++i) {
        std::string tok;
        ls >> tok;
        const size_t colon = tok.find(':');
        if (colon == std::string::npos) continue;
        km.hidden.push_back({uint32_t(std::stoul(tok.substr(0, colon))), std::stoi(tok.substr(colon + 1))});
      }
      c.meta[name] = std::move(km);
    }
    return c;
  }();
  return co;
}

std::string handle_name(const void *handle) {
  Dl_info info{};
  if (!dladdr(handle, &info) || !info.dli_sname || info.dli_saddr != handle) return std::string();
  return info.dli_sname;
}

struct AqlKernel {
  uint64_t object = 0;
  uint32_t kernarg_size = 0, kernarg_align = 16, group_size = 0, private_size = 0;
  KernelMeta meta;
};

// Per-agent state for the process lifetime: the loaded executable and resolved kernels.
struct Agent {
  hsa_agent_t gpu{}, cpu{};
  hsa_executable_t exe{};
  hsa_code_object_reader_t reader{};
  uint32_t queue_max = 0;
  std::mutex mu;
  std::map<const void *, AqlKernel> kernels;
};

struct AgentSearch {
  uint32_t want_bdf = 0, want_domain = 0;
  bool by_pci = false;
  int nth = 0, seen = 0;
  hsa_agent_t gpu{}, cpu{};
  bool have_gpu = false, have_cpu = false;
};

hsa_status_t visit_agent(hsa_agent_t a, void *data) {
  auto *s = static_cast<AgentSearch *>(data);
  hsa_device_type_t t;
  if (hsa_agent_get_info(a, HSA_AGENT_INFO_DEVICE, &t) != HSA_STATUS_SUCCESS) return HSA_STATUS_SUCCESS;
  if (t == HSA_DEVICE_TYPE_CPU && !s->have_cpu) {
    s->cpu = a;
    s->have_cpu = true;
  } else if (t == HSA_DEVICE_TYPE_GPU && !s->have_gpu) {
    uint32_t bdf = 0, dom = 0;
    const bool pci = hsa_agent_get_info(a, hsa_agent_info_t(HSA_AMD_AGENT_INFO_BDFID), &bdf) == HSA_STATUS_SUCCESS &&
                     hsa_agent_get_info(a, hsa_agent_info_t(HSA_AMD_AGENT_INFO_DOMAIN), &dom) == HSA_STATUS_SUCCESS;
    const bool hit = s->by_pci ? (pci && bdf == s->want_bdf && dom == s->want_domain) : s->seen == s->nth;
    ++s->seen;
    if (hit) {
      s->gpu = a;
      s->have_gpu = true;
    }
  }
  return HSA_STATUS_SUCCESS;
}

Agent &agent_for(int device) {
  static std::mutex mu;
  static std::map<int, std::unique_ptr<Agent>> agents;
  std::lock_guard<std::mutex> lk(mu);
  auto it = agents.find(device);
  if (it != agents.end()) return *it->second;
  const CodeObject &co = code_object();
  if (!co.error.empty()) fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: " + co.error);
  PSC_HSA(hsa_init());
  // the HIP device's PCI location names its HSA agent
  AgentSearch s;
  int bus = 0, dev = 0, dom = 0;
  if (hipDeviceGetAttribute(&bus, hipDeviceAttributePciBusId, device) == hipSuccess &&
      hipDeviceGetAttribute(&dev, hipDeviceAttributePciDeviceId, device) == hipSuccess &&
      hipDeviceGetAttribute(&dom, hipDeviceAttributePciDomainID, device) == hipSuccess) {
    s.by_pci = true;
    s.want_bdf = uint32_t(bus) << 8 | uint32_t(dev) << 3;
    s.want_domain = uint32_t(dom);
  } else {
    (void)hipGetLastError();
    s.nth = device;
  }
  PSC_HSA(hsa_iterate_agents(visit_agent, &s));
  if (!s.have_gpu && s.by_pci) {  // no PCI match: fall back to enumeration order
    AgentSearch t;
    t.nth = device;
    PSC_HSA(hsa_iterate_agents(visit_agent, &t));
    s = t;
  }
  if (!s.have_gpu || !s.have_cpu) fail(PSC_ERR_HIP, "AQL dispatch: no HSA agent for HIP device " + std::to_string(device));
  auto a = std::make_unique<Agent>();
  a->gpu = s.gpu;
  a->cpu = s.cpu;
  PSC_HSA(hsa_agent_get_info(a->gpu, HSA_AGENT_INFO_QUEUE_MAX_SIZE, &a->queue_max));
  hsa_profile_t prof;
  PSC_HSA(hsa_agent_get_info(a->gpu, HSA_AGENT_INFO_PROFILE, &prof));
  PSC_HSA(hsa_code_object_reader_create_from_memory(co.bytes.data(), co.bytes.size(), &a->reader));
  PSC_HSA(hsa_executable_create_alt(prof, HSA_DEFAULT_FLOAT_ROUNDING_MODE_DEFAULT, nullptr, &a->exe));
  PSC_HSA(hsa_executable_load_agent_code_object(a->exe, a->gpu, a->reader, nullptr, nullptr));
  PSC_HSA(hsa_executable_freeze(a->exe, nullptr));
  Agent &ref = *a;
  agents[device] = std::move(a);
  return ref;
}

bool meta_supported(const KernelMeta &m, std::string *why, const std::string &name) {
  for (const auto &h : m.hidden)
    if (h.second == kHidUnknown) {
      if (why) *why = "kernel " + name + " needs an implicit argument the AQL dispatcher does not fill";
      return false;
    }
  return true;
}

const AqlKernel &resolve(Agent &ag, const Launch &L) {
  std::lock_guard<std::mutex> lk(ag.mu);
  auto it = ag.kernels.find(L.func);
  if (it != ag.kernels.end()) return it->second;
  const std::string name = handle_name(L.func);
  if (name.empty()) fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: a kernel handle has no exported name");
  const CodeObject &co = code_object();
  auto m = co.meta.find(name);
  if (m == co.meta.end()) fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: kernel " + name + " is not in the argument table");
  std::string why;
  if (!meta_supported(m->second, &why, name)) fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: " + why);
  hsa_executable_symbol_t sym;
  PSC_HSA(hsa_executable_get_symbol_by_name(ag.exe, (name + ".kd").c_str(), &ag.gpu, &sym));
  AqlKernel k;
  k.meta = m->second;
  PSC_HSA(hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_OBJECT, &k.object));
  PSC_HSA(hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_KERNARG_SEGMENT_SIZE, &k.kernarg_size));
  PSC_HSA(hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_KERNARG_SEGMENT_ALIGNMENT,
                                         &k.kernarg_align));
  PSC_HSA(hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_GROUP_SEGMENT_SIZE, &k.group_size));
  PSC_HSA(hsa_executable_symbol_get_info(sym, HSA_EXECUTABLE_SYMBOL_INFO_KERNEL_PRIVATE_SEGMENT_SIZE, &k.private_size));
  if (k.meta.explicit_bytes > sizeof(L.args) || k.meta.explicit_bytes > k.kernarg_size)
    fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: argument record of " + name + " does not fit");
  for (const auto &h : k.meta.hidden)
    if (h.first + 8 > k.kernarg_size) fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: implicit argument outside the segment");
  return ag.kernels.emplace(L.func, std::move(k)).first->second;
}

// The kernel argument segment of one launch: the explicit record, then the implicit arguments.
void fill_kernarg(const AqlKernel &k, const Launch &L, unsigned char *seg) {
  std::memset(seg, 0, k.kernarg_size);
  std::memcpy(seg, L.args, k.meta.explicit_bytes);
  const uint32_t bc[3] = {L.grid.x, L.grid.y, L.grid.z};
  const uint32_t gs[3] = {L.block.x, L.block.y, L.block.z};
  for (const auto &h : k.meta.hidden) {
    unsigned char *p = seg + h.first;
    auto put32 = [&](uint32_t v) { std::memcpy(p, &v, 4); };
    auto put16 = [&](uint16_t v) { std::memcpy(p, &v, 2); };
    switch (h.second) {
      case kBlockCountX: case kBlockCountY: case kBlockCountZ: put32(bc[h.second - kBlockCountX]); break;
      case kGroupSizeX: case kGroupSizeY: case kGroupSizeZ: put16(uint16_t(gs[h.second - kGroupSizeX])); break;
      case kRemainderX: case kRemainderY: case kRemainderZ: put16(0); break;   // whole work-groups only
      case kGlobalOffsetX: case kGlobalOffsetY: case kGlobalOffsetZ: break;   // zero
      case kGridDims: put16(3); break;
      default: break;
    }
  }
}

constexpr uint16_t kScopeShiftA = HSA_PACKET_HEADER_SCACQUIRE_FENCE_SCOPE;
constexpr uint16_t kScopeShiftR = HSA_PACKET_HEADER_SCRELEASE_FENCE_SCOPE;

// barrier: the packet starts only after every earlier packet of its queue has completed (the
// in-order queue); without it a dispatch may start while earlier ones still run
uint16_t header(hsa_packet_type_t type, hsa_fence_scope_t acq, hsa_fence_scope_t rel, bool barrier = true) {
  return uint16_t(type << HSA_PACKET_HEADER_TYPE) | uint16_t((barrier ? 1 : 0) << HSA_PACKET_HEADER_BARRIER) |
         uint16_t(acq << kScopeShiftA) | uint16_t(rel << kScopeShiftR);
}

std::atomic<uint32_t> g_queue_error{0};

void queue_error(hsa_status_t status, hsa_queue_t *, void *) {
  g_queue_error.store(uint32_t(status) ? uint32_t(status) : 1u, std::memory_order_relaxed);
}

}  // namespace

bool aql_launch_supported(const Launch &L, std::string *why) {
  const CodeObject &co = code_object();
  if (!co.error.empty()) {
    if (why) *why = co.error;
    return false;
  }
  const std::string name = handle_name(L.func);
  if (name.empty()) {
    if (why) *why = "kernel handle has no exported name";
    return false;
  }
  auto m = co.meta.find(name);
  if (m == co.meta.end()) {
    if (why) *why = "kernel " + name + " is not in the argument table";
    return false;
  }
  if (m->second.explicit_bytes > sizeof(L.args)) {
    if (why) *why = "argument record of " + name + " does not fit";
    return false;
  }
  return meta_supported(m->second, why, name);
}

struct AqlSchedule::Impl {
  int device = 0;
  Agent *ag = nullptr;
  const SchedPlan *plan = nullptr;
  bool record = false;
  std::vector<hsa_queue_t *> queues;       // per stream; nullptr for streams without kernels
  std::vector<hsa_signal_t> sig;           // per op: its completion
  hsa_signal_t start_sig{}, end_sig{};
  std::vector<const AqlKernel *> kern;     // per op: the kernel, nullptr for copies and empty launches
  std::vector<uint64_t> kernarg_off;       // per op, offset of its segment in `kernargs`
  std::vector<Launch> launches;            // per op (kernels)
  std::vector<const AqlKernel *> mark_kern;  // per op: a component mark after it, or nullptr
  std::vector<uint64_t> mark_off;
  std::vector<Launch> marks;
  std::vector<char> acq_sys, rel_sys;      // per op: system-scope fences where kernels meet copies
  bool ooo = false;                        // out-of-order queues (plan.out_of_order)
  std::vector<hsa_signal_t> qend;          // out of order: per queue, completes after all its packets
  std::vector<std::vector<char>> covered;  // out of order, per run: per queue, ops already awaited there
  const AqlKernel *clock_kern = nullptr;   // start and end clock marks
  Launch clock_launch[2];
  uint64_t clock_off[2] = {0, 0};
  const AqlKernel *cstart_kern = nullptr;  // component start mark (mark_components)
  Launch cstart_launch;
  uint64_t cstart_off = 0;
  void *kernargs = nullptr;                // device memory
  uint64_t *clocks = nullptr;              // page-locked: start and end clock
  double clock_mhz = 100.0;
  bool running = false;
  // per run
  std::vector<AqlCopy> copies;
  std::vector<std::vector<hsa_signal_t>> pending;  // per stream: dependencies of its next op
  std::vector<hsa_signal_t> tail;                  // per stream: completion of its last op
  std::vector<char> tail_copy;                     // per stream: its last op was a copy
  std::vector<char> dispatched;                    // per op: handed to a queue or a DMA engine
  std::vector<int32_t> pkt_count;                  // per stream

  // Waits up to `ms` milliseconds for the end mark.
  bool ended_within(int ms) const {
    const auto t0 = std::chrono::steady_clock::now();
    while (hsa_signal_load_scacquire(end_sig) != 0) {
      if (std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(ms)) return false;
      std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
    return true;
  }

  ~Impl() {
    bool drained = true;
    if (running && end_sig.handle && !ended_within(60000)) {
      // a run that cannot finish (an op's signal never completes): complete every signal from the
      // host so the queues drain, then give them a last bound; queues that still hold work are
      // left in place rather than torn down under the command processor
      for (hsa_signal_t x : sig)
        if (x.handle) hsa_signal_store_screlease(x, 0);
      if (start_sig.handle) hsa_signal_store_screlease(start_sig, 0);
      drained = ended_within(10000);
    }
    if (!drained) return;
    for (hsa_queue_t *q : queues)
      if (q) (void)hsa_queue_destroy(q);
    for (hsa_signal_t x : sig)
      if (x.handle) (void)hsa_signal_destroy(x);
    for (hsa_signal_t x : qend)
      if (x.handle) (void)hsa_signal_destroy(x);
    if (start_sig.handle) (void)hsa_signal_destroy(start_sig);
    if (end_sig.handle) (void)hsa_signal_destroy(end_sig);
    if (kernargs) (void)hipFree(kernargs);
    if (clocks) (void)hipHostFree(clocks);
  }

  // Writes n packets on `stream`'s queue: bodies first, then the headers in order (the command
  // processor starts on a packet once its header is valid), then one doorbell.
  template <typename F>
  void write(int32_t stream, int n, const uint16_t *hdr, const uint16_t *setup, F &&fill) {
    hsa_queue_t *qu = queues[stream];
    const uint64_t first = hsa_queue_add_write_index_relaxed(qu, uint64_t(n));
    const uint64_t size = qu->size;
    // the ring holds a whole run (sized at set-up), so this waits at most for the previous run's tail
    while (first + uint64_t(n) - hsa_queue_load_read_index_scacquire(qu) > size) PSC_AQL_PAUSE();
    auto *base = static_cast<hsa_kernel_dispatch_packet_t *>(qu->base_address);
    for (int i = 0; i < n; ++i) fill(i, &base[(first + uint64_t(i)) & (size - 1)]);
    for (int i = 0; i < n; ++i)
      __atomic_store_n(reinterpret_cast<uint32_t *>(&base[(first + uint64_t(i)) & (size - 1)]),
                       uint32_t(hdr[i]) | (uint32_t(setup[i]) << 16), __ATOMIC_RELEASE);
    hsa_signal_store_screlease(qu->doorbell_signal, hsa_signal_value_t(first + uint64_t(n) - 1));
    pkt_count[stream] += n;
  }

  void dispatch_body(hsa_kernel_dispatch_packet_t *p, const AqlKernel &k, const Launch &L, uint64_t off,
                     hsa_signal_t s) const {
    p->workgroup_size_x = uint16_t(L.block.x);
    p->workgroup_size_y = 1;
    p->workgroup_size_z = 1;
    p->reserved0 = 0;
    p->grid_size_x = L.grid.x * L.block.x;
    p->grid_size_y = 1;
    p->grid_size_z = 1;
    p->private_segment_size = k.private_size;
    p->group_segment_size = k.group_size + L.shmem;
    p->kernel_object = k.object;
    p->kernarg_address = static_cast<char *>(kernargs) + off;
    p->reserved2 = 0;
    p->completion_signal = s;
  }

  // Barrier-AND packets for `deps` (five per packet), then up to two kernel dispatches; `done`
  // completes with the first kernel, or with the last barrier when there is no kernel.
  struct Kd {
    const AqlKernel *k;
    const Launch *L;
    uint64_t off;
    hsa_signal_t done;
    bool acq_sys, rel_sys;
    bool barrier = true;  // wait for every earlier packet of the queue
  };
  // Barrier-AND packets wait for their signals and hold back every later packet of the queue;
  // in an in-order queue they also wait for every earlier packet, in an out-of-order one only
  // when `all_before` asks for it (the queue's closing barrier).
  void emit(int32_t stream, std::vector<hsa_signal_t> &deps, hsa_signal_t done_if_no_kernel, const Kd *kd,
            int nk, bool all_before = false) {
    int nb = int((deps.size() + 4) / 5);
    if (nk == 0 && nb == 0 && done_if_no_kernel.handle) nb = 1;  // a no-op that completes in order
    const int n = nb + nk;
    if (n == 0) return;
    std::vector<uint16_t> H(n), S(n, 0);
    for (int i = 0; i < nb; ++i)
      H[i] = header(HSA_PACKET_TYPE_BARRIER_AND, HSA_FENCE_SCOPE_AGENT, HSA_FENCE_SCOPE_AGENT, !ooo || all_before);
    for (int j = 0; j < nk; ++j) {
      H[nb + j] = header(HSA_PACKET_TYPE_KERNEL_DISPATCH, kd[j].acq_sys ? HSA_FENCE_SCOPE_SYSTEM : HSA_FENCE_SCOPE_AGENT,
                         kd[j].rel_sys ? HSA_FENCE_SCOPE_SYSTEM : HSA_FENCE_SCOPE_AGENT, !ooo || kd[j].barrier);
      S[nb + j] = uint16_t(3 << HSA_KERNEL_DISPATCH_PACKET_SETUP_DIMENSIONS);
    }
    write(stream, n, H.data(), S.data(), [&](int i, hsa_kernel_dispatch_packet_t *pkt) {
      if (i < nb) {
        auto *b = reinterpret_cast<hsa_barrier_and_packet_t *>(pkt);
        b->reserved0 = 0;
        b->reserved1 = 0;
        for (int j = 0; j < 5; ++j) {
          const size_t d = size_t(i) * 5 + size_t(j);
          b->dep_signal[j] = d < deps.size() ? deps[d] : hsa_signal_t{0};
        }
        b->reserved2 = 0;
        b->completion_signal = (nk == 0 && i == nb - 1) ? done_if_no_kernel : hsa_signal_t{0};
      } else {
        const Kd &x = kd[i - nb];
        dispatch_body(pkt, *x.k, *x.L, x.off, x.done);
      }
    });
    deps.clear();
  }

  bool host_memory_ok(const void *p, size_t bytes) const {
    hsa_amd_pointer_info_t info{};
    info.size = sizeof(info);
    if (hsa_amd_pointer_info(const_cast<void *>(p), &info, nullptr, nullptr, nullptr) != HSA_STATUS_SUCCESS)
      return false;
    if (info.type == HSA_EXT_POINTER_TYPE_UNKNOWN || !info.hostBaseAddress) return false;
    const uintptr_t b = reinterpret_cast<uintptr_t>(info.hostBaseAddress), a = reinterpret_cast<uintptr_t>(p);
    return a >= b && a + bytes <= b + info.sizeInBytes;
  }
};

AqlSchedule::AqlSchedule(int device, const SchedPlan &plan, const std::vector<Launch> &launch,
                         const std::vector<Launch> &mark_after, const Launch *mark_start, bool record)
    : p_(new Impl) {
  Impl &I = *p_;
  I.device = device;
  I.plan = &plan;
  I.record = record;
  I.ooo = plan.out_of_order;
  I.ag = &agent_for(device);
  Agent &ag = *I.ag;
  const size_t n = plan.ops.size();
  const int32_t T = plan.total_streams;
  // a queue for every stream holding a kernel (and stream 0, which holds the marks and the join)
  std::vector<char> has_kernel(T, 0);
  has_kernel[0] = 1;
  for (const Op &op : plan.ops)
    if (op.type == PSC_OP_KERNEL) has_kernel[op.stream] = 1;
  // packets per queue per run, an upper bound: start, per op its barriers, dispatch and mark, join
  std::vector<uint64_t> need(T, 6);
  need[0] += uint64_t(T) / 5 + 8;
  for (const Op &op : plan.ops) need[op.stream] += 3 + (op.waits.size() + 1 + 4) / 5;
  I.queues.assign(T, nullptr);
  for (int32_t s = 0; s < T; ++s) {
    if (!has_kernel[s]) continue;
    uint32_t size = 256;
    while (size < need[s] && size < ag.queue_max) size *= 2;
    if (size < need[s]) fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: a stream holds more packets than a queue");
    PSC_HSA(hsa_queue_create(ag.gpu, size, HSA_QUEUE_TYPE_SINGLE, queue_error, nullptr, UINT32_MAX, UINT32_MAX,
                             &I.queues[s]));
    if (record) PSC_HSA(hsa_amd_profiling_set_profiler_enabled(I.queues[s], 1));
  }
  if (record) PSC_HSA(hsa_amd_profiling_async_copy_enable(true));
  I.sig.assign(n, hsa_signal_t{0});
  for (size_t o = 0; o < n; ++o) PSC_HSA(hsa_amd_signal_create(1, 0, nullptr, HSA_AMD_SIGNAL_AMD_GPU_ONLY, &I.sig[o]));
  PSC_HSA(hsa_amd_signal_create(1, 0, nullptr, HSA_AMD_SIGNAL_AMD_GPU_ONLY, &I.start_sig));
  if (I.ooo) {
    I.qend.assign(T, hsa_signal_t{0});
    for (int32_t s = 0; s < T; ++s)
      if (I.queues[s]) PSC_HSA(hsa_amd_signal_create(1, 0, nullptr, HSA_AMD_SIGNAL_AMD_GPU_ONLY, &I.qend[s]));
  }
  PSC_HSA(hsa_signal_create(1, 0, nullptr, &I.end_sig));
  // kernel argument segments in one device block, written once
  I.kern.assign(n, nullptr);
  I.mark_kern.assign(n, nullptr);
  I.kernarg_off.assign(n, 0);
  I.mark_off.assign(n, 0);
  I.launches.assign(n, Launch{});
  I.marks.assign(n, Launch{});
  uint64_t total = 0;
  auto take = [&](const AqlKernel &k) {
    const uint64_t a = std::max<uint64_t>(64, k.kernarg_align);
    total = (total + a - 1) / a * a;
    const uint64_t off = total;
    total += k.kernarg_size;
    return off;
  };
  auto check_shape = [](const Launch &L) {
    const uint64_t items = uint64_t(L.grid.x) * L.block.x;
    if (items > 0xffffffffull || L.grid.y != 1 || L.grid.z != 1 || L.block.y != 1 || L.block.z != 1 ||
        L.block.x == 0 || L.block.x > 1024)
      fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: launch shape outside one 32-bit dimension");
  };
  for (size_t o = 0; o < n; ++o) {
    const Op &op = plan.ops[o];
    if (op.type != PSC_OP_KERNEL) continue;
    const Launch &L = launch[op.kernel];
    I.launches[o] = L;
    if (!L.empty) {
      check_shape(L);
      I.kern[o] = &resolve(ag, L);
      I.kernarg_off[o] = take(*I.kern[o]);
    }
    if (op.kernel < int32_t(mark_after.size()) && mark_after[op.kernel].func) {
      I.marks[o] = mark_after[op.kernel];
      I.mark_kern[o] = &resolve(ag, I.marks[o]);
      I.mark_off[o] = take(*I.mark_kern[o]);
    }
  }
  PSC_HIPA(hipSetDevice(device));
  PSC_HIPA(hipHostMalloc(reinterpret_cast<void **>(&I.clocks), 64, hipHostMallocDefault));
  I.clocks[0] = I.clocks[1] = 0;
  make_mark(I.clock_launch[0], I.clocks);
  make_mark(I.clock_launch[1], I.clocks + 1);
  I.clock_kern = &resolve(ag, I.clock_launch[0]);
  I.clock_off[0] = take(*I.clock_kern);
  I.clock_off[1] = take(*I.clock_kern);
  if (mark_start && mark_start->func) {
    I.cstart_launch = *mark_start;
    I.cstart_kern = &resolve(ag, I.cstart_launch);
    I.cstart_off = take(*I.cstart_kern);
  }
  std::vector<unsigned char> host(std::max<uint64_t>(total, 64), 0);
  for (size_t o = 0; o < n; ++o) {
    if (I.kern[o]) fill_kernarg(*I.kern[o], I.launches[o], host.data() + I.kernarg_off[o]);
    if (I.mark_kern[o]) fill_kernarg(*I.mark_kern[o], I.marks[o], host.data() + I.mark_off[o]);
  }
  for (int i = 0; i < 2; ++i) fill_kernarg(*I.clock_kern, I.clock_launch[i], host.data() + I.clock_off[i]);
  if (I.cstart_kern) fill_kernarg(*I.cstart_kern, I.cstart_launch, host.data() + I.cstart_off);
  PSC_HIPA(hipMalloc(&I.kernargs, host.size()));
  PSC_HIPA(hipMemcpy(I.kernargs, host.data(), host.size(), hipMemcpyHostToDevice));
  // system-scope fences where a kernel meets a copy: the DMA engines read and write memory, not
  // the GPU's caches
  I.acq_sys.assign(n, 0);
  I.rel_sys.assign(n, 0);
  std::vector<int32_t> prev(n, -1), last(T, -1);
  for (size_t o = 0; o < n; ++o) {
    prev[o] = last[plan.ops[o].stream];
    last[plan.ops[o].stream] = int32_t(o);
  }
  for (size_t o = 0; o < n; ++o) {
    const Op &op = plan.ops[o];
    const bool copy = op.type != PSC_OP_KERNEL;
    std::vector<int32_t> before(op.waits.begin(), op.waits.end());
    if (prev[o] >= 0) before.push_back(prev[o]);
    for (int32_t w : before) {
      if (copy) I.rel_sys[w] = 1;
      if (plan.ops[w].type != PSC_OP_KERNEL) I.acq_sys[o] = 1;
    }
  }
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) == hipSuccess && khz > 0)
    I.clock_mhz = khz / 1000.0;
  else
    (void)hipGetLastError();
}

AqlSchedule::~AqlSchedule() = default;

void AqlSchedule::begin(const std::vector<AqlCopy> &copies) {
  Impl &I = *p_;
  const SchedPlan &plan = *I.plan;
  const size_t n = plan.ops.size();
  const int32_t T = plan.total_streams;
  if (copies.size() != n) fail(PSC_ERR_ARG, "AQL dispatch: copy list does not match the schedule");
  // every check before the first packet: a run is either fully enqueued or not at all
  for (size_t o = 0; o < n; ++o) {
    const AqlCopy &c = copies[o];
    if (plan.ops[o].type == PSC_OP_KERNEL || !c.active) continue;
    const void *host = c.h2d ? c.src : c.dst;
    const size_t hpitch = c.h2d ? c.spitch : c.dpitch;
    const size_t span = hpitch * (c.height - 1) + c.width;
    if (!I.host_memory_ok(host, span))
      fail(PSC_ERR_ARG, "AQL dispatch copies from and to page-locked host memory only (psc_host_alloc)");
    const bool dense = c.dpitch == c.width && c.spitch == c.width;
    const bool al4 = reinterpret_cast<uintptr_t>(c.dst) % 4 == 0 && reinterpret_cast<uintptr_t>(c.src) % 4 == 0 &&
                     c.dpitch % 4 == 0 && c.spitch % 4 == 0 && c.width % 4 == 0;
    if (!dense && !al4)
      fail(PSC_ERR_UNSUPPORTED, "AQL dispatch: a strided copy is not 4-byte aligned (the DMA engine's rule)");
  }
  if (uint32_t e = g_queue_error.load()) fail(PSC_ERR_HIP, "AQL queue error " + std::to_string(e));
  I.copies = copies;
  for (size_t o = 0; o < n; ++o) {
    const bool inactive_copy = plan.ops[o].type != PSC_OP_KERNEL && !copies[o].active;
    hsa_signal_store_relaxed(I.sig[o], inactive_copy ? 0 : 1);   // nothing to wait for on a skipped copy
  }
  hsa_signal_store_relaxed(I.start_sig, 1);
  hsa_signal_store_relaxed(I.end_sig, 1);
  for (hsa_signal_t x : I.qend)
    if (x.handle) hsa_signal_store_relaxed(x, 1);
  if (I.ooo) I.covered.assign(T, std::vector<char>(n, 0));
  I.clocks[0] = I.clocks[1] = 0;
  I.pending.assign(T, {});
  I.tail.assign(T, I.start_sig);
  I.tail_copy.assign(T, 1);   // every stream starts behind the start mark
  I.dispatched.assign(n, 0);
  I.pkt_count.assign(T, 0);
  I.running = true;
  // queue 0: the start clock (and the component start mark), whose completion every stream waits for
  std::vector<hsa_signal_t> none;
  Impl::Kd k0[2] = {{I.clock_kern, &I.clock_launch[0], I.clock_off[0],
                     I.cstart_kern ? hsa_signal_t{0} : I.start_sig, false, true},
                    {I.cstart_kern, &I.cstart_launch, I.cstart_off, I.start_sig, false, false}};
  I.emit(0, none, hsa_signal_t{0}, k0, I.cstart_kern ? 2 : 1);
  if (I.ooo) {
    // the marks do not hold back later dispatches of an out-of-order queue: wait for them
    std::vector<hsa_signal_t> d{I.start_sig};
    I.emit(0, d, hsa_signal_t{0}, nullptr, 0);
  }
  I.tail_copy[0] = 0;
  for (int32_t s = 1; s < T; ++s)
    if (I.queues[s]) {
      std::vector<hsa_signal_t> d{I.start_sig};
      I.emit(s, d, hsa_signal_t{0}, nullptr, 0);
      I.tail_copy[s] = 0;
    }
}

void AqlSchedule::wait(int32_t op, int32_t awaited) {
  Impl &I = *p_;
  const Op &a = I.plan->ops[awaited];
  if (a.type != PSC_OP_KERNEL && !I.copies[awaited].active) return;   // a skipped copy
  const int32_t s = I.plan->ops[op].stream;
  if (I.ooo && I.plan->ops[op].type == PSC_OP_KERNEL) {
    // a barrier-AND holds back every later packet of its queue, so an op awaited once there is
    // complete for everything after it
    if (I.covered[s][awaited]) return;
    I.covered[s][awaited] = 1;
  }
  I.pending[s].push_back(I.sig[awaited]);
}

void AqlSchedule::exec(int32_t o) {
  Impl &I = *p_;
  const Op &op = I.plan->ops[o];
  const int32_t s = op.stream;
  std::vector<hsa_signal_t> &deps = I.pending[s];
  if (op.type == PSC_OP_KERNEL) {
    if (I.tail_copy[s] && !I.ooo) deps.push_back(I.tail[s]);
    // a component mark that follows the kernel carries the op's completion, so the end of the run
    // (which waits for every stream's last op) also waits for the mark
    Impl::Kd kd[2];
    int nk = 0;
    const bool mark = I.mark_kern[o] != nullptr;
    if (I.kern[o])
      kd[nk++] = {I.kern[o], &I.launches[o], I.kernarg_off[o], mark ? hsa_signal_t{0} : I.sig[o], I.acq_sys[o] != 0,
                  I.rel_sys[o] != 0, false};
    // a mark stamps the clock after its kernel: in an out-of-order queue it waits for every
    // earlier packet (its kernel included)
    if (mark) kd[nk++] = {I.mark_kern[o], &I.marks[o], I.mark_off[o], I.sig[o], false, I.rel_sys[o] != 0, true};
    I.emit(s, deps, I.sig[o], kd, nk);
    I.tail[s] = I.sig[o];
    I.tail_copy[s] = 0;
    I.dispatched[o] = 1;
    return;
  }
  const AqlCopy &c = I.copies[o];
  if (!c.active) {
    // a skipped copy keeps its stream position: its waits pass to the stream's next op, since
    // the planner leaves out waits of later ops that this op's waits already imply
    I.dispatched[o] = 1;
    return;
  }
  deps.push_back(I.tail[s]);
  const hsa_agent_t gpu = I.ag->gpu, cpu = I.ag->cpu;
  if (c.dpitch == c.width && c.spitch == c.width) {
    PSC_HSA(hsa_amd_memory_async_copy(c.dst, c.h2d ? gpu : cpu, c.src, c.h2d ? cpu : gpu, c.width * c.height,
                                      uint32_t(deps.size()), deps.data(), I.sig[o]));
  } else {
    hsa_pitched_ptr_t dp{c.dst, c.dpitch, c.dpitch * c.height};
    hsa_pitched_ptr_t sp{const_cast<void *>(c.src), c.spitch, c.spitch * c.height};
    const hsa_dim3_t zero{0, 0, 0}, range{uint32_t(c.width), uint32_t(c.height), 1};
    PSC_HSA(hsa_amd_memory_async_copy_rect(&dp, &zero, &sp, &zero, &range, gpu,
                                           c.h2d ? hsaHostToDevice : hsaDeviceToHost, uint32_t(deps.size()),
                                           deps.data(), I.sig[o]));
  }
  deps.clear();
  I.tail[s] = I.sig[o];
  I.tail_copy[s] = 1;
  I.dispatched[o] = 1;
}

void AqlSchedule::release_undispatched() {
  Impl &I = *p_;
  for (size_t o = 0; o < I.dispatched.size(); ++o)
    if (!I.dispatched[o]) hsa_signal_store_screlease(I.sig[o], 0);
  for (auto &d : I.pending) d.clear();
}

void AqlSchedule::end() {
  Impl &I = *p_;
  const int32_t T = I.plan->total_streams;
  std::vector<hsa_signal_t> deps;
  if (I.ooo) {
    // a queue's last packet says nothing about its earlier kernels: each queue ends with a
    // barrier over all of its packets, and the end mark waits for those
    for (int32_t s = 1; s < T; ++s)
      if (I.queues[s]) {
        std::vector<hsa_signal_t> none;
        I.emit(s, none, I.qend[s], nullptr, 0, true);
        deps.push_back(I.qend[s]);
      } else if (I.tail[s].handle != I.start_sig.handle) {
        deps.push_back(I.tail[s]);   // a copy stream: in order
      }
  } else {
    for (int32_t s = 1; s < T; ++s)
      if (I.tail[s].handle != I.start_sig.handle) deps.push_back(I.tail[s]);
  }
  if (I.tail_copy[0] && I.tail[0].handle != I.start_sig.handle) deps.push_back(I.tail[0]);
  Impl::Kd k1{I.clock_kern, &I.clock_launch[1], I.clock_off[1], I.end_sig, true, true};
  I.emit(0, deps, hsa_signal_t{0}, &k1, 1);
  packets_ = 0;
  for (int32_t c : I.pkt_count) packets_ += c;
}

bool AqlSchedule::wait_end(int timeout_ms) {
  Impl &I = *p_;
  const auto t0 = std::chrono::steady_clock::now();
  uint32_t spins = 0;
  while (hsa_signal_load_scacquire(I.end_sig) != 0) {
    if (uint32_t e = g_queue_error.load(std::memory_order_relaxed))
      fail(PSC_ERR_HIP, "AQL queue error " + std::to_string(e));
    if (++spins % 1024 == 0) {
      const auto el = std::chrono::steady_clock::now() - t0;
      if (timeout_ms > 0 && el > std::chrono::milliseconds(timeout_ms)) return false;
      if (el > std::chrono::milliseconds(2)) std::this_thread::yield();
    }
    PSC_AQL_PAUSE();
  }
  I.running = false;
  return true;
}

double AqlSchedule::makespan_ms() const {
  const Impl &I = *p_;
  return double(int64_t(I.clocks[1] - I.clocks[0])) / I.clock_mhz / 1000.0;
}

void AqlSchedule::op_times(std::vector<float> &start_us, std::vector<float> &end_us) const {
  const Impl &I = *p_;
  if (!I.record) fail(PSC_ERR_STATE, "AQL schedule was not prepared with record_ops");
  const size_t n = I.plan->ops.size();
  start_us.assign(n, 0.f);
  end_us.assign(n, 0.f);
  // dispatch and copy times both come in the HSA system clock domain (no tick conversion)
  uint64_t freq = 0;
  PSC_HSA(hsa_system_get_info(HSA_SYSTEM_INFO_TIMESTAMP_FREQUENCY, &freq));
  const double us_per_tick = 1e6 / double(freq ? freq : 1);
  hsa_amd_profiling_dispatch_time_t t0{};
  PSC_HSA(hsa_amd_profiling_get_dispatch_time(I.ag->gpu, I.start_sig, &t0));
  const uint64_t base = t0.end;
  auto rel = [&](uint64_t v) { return float((double(int64_t(v - base))) * us_per_tick); };
  for (size_t o = 0; o < n; ++o) {
    const Op &op = I.plan->ops[o];
    if (op.type == PSC_OP_KERNEL) {
      if (!I.kern[o]) continue;
      hsa_amd_profiling_dispatch_time_t t{};
      PSC_HSA(hsa_amd_profiling_get_dispatch_time(I.ag->gpu, I.sig[o], &t));
      start_us[o] = rel(t.start);
      end_us[o] = rel(t.end);
    } else if (I.copies[o].active) {
      hsa_amd_profiling_async_copy_time_t t{};
      PSC_HSA(hsa_amd_profiling_get_async_copy_time(I.sig[o], &t));
      start_us[o] = rel(t.start);
      end_us[o] = rel(t.end);
    }
  }
}

}  // namespace psc
