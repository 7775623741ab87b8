// Host-to-device upload of the small per-call tables (descriptors, orbital
// energies, work items, contraction lists) without blocking the host.
//
// A copy from pageable host memory is synchronous in HIP, so the tables are
// first written into one of a few page-locked host buffers owned by the
// library; the copies from there are stream-ordered and return at once.  A
// buffer is reused only after the event recorded behind its last copies has
// completed, so the host waits only when it runs more than kSlots calls
// ahead of the device.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <string>
#include <vector>

namespace sie {

// One page-locked buffer and the event behind its last copies.
struct StagingSlot {
  void* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  int dev = -1;
  bool pending = false;
};

class Staging {
 public:
  static constexpr int kSlots = 4;

  // One call's uploads: add() copies bytes into the slot and queues the
  // device destination; commit() enqueues the copies on `s` and records the
  // slot's event.  The ring stays locked from begin() to commit() (or the
  // destructor), so concurrent calls never share a slot.
  class Batch {
   public:
    ~Batch() {
      if (lock_.owns_lock()) lock_.unlock();
    }
    void add(void* dst, const void* src, size_t bytes) {
      if (bytes == 0) return;
      std::memcpy(static_cast<char*>(slot_->host) + used_, src, bytes);
      parts_.push_back({dst, used_, bytes});
      used_ += (bytes + 255) / 256 * 256;
    }
    hipError_t commit(hipStream_t s) {
      hipError_t e = hipSuccess;
      for (const Part& p : parts_) {
        e = hipMemcpyAsync(p.dst, static_cast<char*>(slot_->host) + p.off, p.bytes,
                           hipMemcpyHostToDevice, s);
        if (e != hipSuccess) break;
      }
      if (e == hipSuccess) e = hipEventRecord(slot_->done, s);
      slot_->pending = e == hipSuccess;
      lock_.unlock();
      return e;
    }

   private:
    friend class Staging;
    struct Part {
      void* dst;
      size_t off, bytes;
    };
    StagingSlot* slot_ = nullptr;
    std::unique_lock<std::mutex> lock_;
    std::vector<Part> parts_;
    size_t used_ = 0;
  };

  // Reserves a slot of at least `bytes` (sum of the add() sizes rounded up to
  // 256 each) on the current device.
  hipError_t begin(size_t bytes, Batch& b) {
    b.lock_ = std::unique_lock<std::mutex>(mu_);
    StagingSlot& sl = slots_[next_];
    next_ = (next_ + 1) % kSlots;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (sl.pending) {      // the slot's previous copies must have landed
      e = hipEventSynchronize(sl.done);
      if (e != hipSuccess) return e;
      sl.pending = false;
    }
    if (sl.done && sl.dev != dev) {
      (void)hipEventDestroy(sl.done);
      sl.done = nullptr;
    }
    if (!sl.done) {
      e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
      if (e != hipSuccess) return e;
      sl.dev = dev;
    }
    if (sl.cap < bytes) {
      if (sl.host) (void)hipHostFree(sl.host);
      sl.host = nullptr;
      sl.cap = 0;
      const size_t cap = bytes < (size_t(1) << 20) ? (size_t(1) << 20) : bytes + bytes / 4;
      e = hipHostMalloc(&sl.host, cap, hipHostMallocPortable);
      if (e != hipSuccess) return e;
      sl.cap = cap;
    }
    b.slot_ = &sl;
    b.parts_.clear();
    b.used_ = 0;
    return hipSuccess;
  }

  static size_t padded(size_t bytes) { return (bytes + 255) / 256 * 256; }

 private:
  std::mutex mu_;
  StagingSlot slots_[kSlots];
  int next_ = 0;
};

}  // namespace sie
