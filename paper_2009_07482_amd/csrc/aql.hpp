// Dispatch through the GPU's own command queues: every stream of a schedule is an HSA user-mode
// queue (an AQL ring the command processor reads), every kernel an AQL dispatch packet written
// by the host, every event precedence a completion signal that a barrier-AND packet on the
// consuming queue waits for, and every host copy an SDMA transfer whose dependencies are the same
// signals.  This is the command-queue model of the paper (Sec. III, Def. 4: in-order queues plus
// cross-queue precedences) at the level the hardware exposes it, without the HIP runtime's
// per-launch cost (~2.5 us of host time per launch and per event record).
//
// Kernels come from the library's own gfx950 code object (libpsc_kernels.hsaco, extracted at
// build time from the same fat binary the HIP path loads) and are found by the name of their host
// handle; libpsc_kernels.kargs lists, per kernel, the size of its explicit argument record and the
// offsets of the implicit (hidden) arguments the compiler asked for, which the host fills per
// packet.
#pragma once

#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "core.hpp"
#include "kernels.hpp"

namespace psc {

// A host copy of one op, resolved against the caller's host memory.
struct AqlCopy {
  bool active = false;
  bool h2d = true;
  void *dst = nullptr;
  const void *src = nullptr;
  size_t dpitch = 0, spitch = 0, width = 0, height = 0;
};

class AqlSchedule {
 public:
  // Resolves every launch in the library's code object on `device`, creates one queue per
  // stream that holds a kernel, one completion signal per op and the kernel argument records
  // (device memory, written once).  mark_after[k] (may be empty) is a launch that follows kernel
  // k's op and mark_start (may be NULL) one that precedes every op (component completion marks).
  // record: per-op timestamps from the queues' profiler and the DMA engines.
  AqlSchedule(int device, const SchedPlan &plan, const std::vector<Launch> &launch,
              const std::vector<Launch> &mark_after, const Launch *mark_start, bool record);
  ~AqlSchedule();
  AqlSchedule(const AqlSchedule &) = delete;
  AqlSchedule &operator=(const AqlSchedule &) = delete;

  // One run: begin() resets the signals and starts every queue behind a start mark; the
  // dispatcher then calls wait / exec per op (from any thread, each stream from one thread);
  // end() joins every stream into queue 0 behind an end mark.
  void begin(const std::vector<AqlCopy> &copies);
  void wait(int32_t op, int32_t awaited);
  void exec(int32_t op);
  void end();
  // After a failed enqueue: completes the signals of every op not handed to the GPU, so the
  // queues drain once end() is enqueued.
  void release_undispatched();
  // Waits for the end mark (timeout_ms <= 0: without limit); false on timeout.
  bool wait_end(int timeout_ms);
  double makespan_ms() const;          // end mark - start mark, device wall clock
  // Per-op (start, end) in microseconds after the start mark (record mode only).
  void op_times(std::vector<float> &start_us, std::vector<float> &end_us) const;
  int32_t packets_last_run() const { return packets_; }

 private:
  struct Impl;
  std::unique_ptr<Impl> p_;
  int32_t packets_ = 0;
};

// Host-only: whether the code object metadata describes every kernel this launch can use (the
// kernel's host handle has a name, the name is listed and its implicit arguments are all of the
// kinds the host fills).  Sets *why on failure.
bool aql_launch_supported(const Launch &L, std::string *why);

}  // namespace psc
