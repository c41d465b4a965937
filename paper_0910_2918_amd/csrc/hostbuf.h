// Pinned host memory for the host side of the library (no device code).
#pragma once

#include <cstddef>

namespace nk {

// Pinned host memory mapped into the device's address space (fine-grained):
// kernels write small results straight into it, so the host reads them
// without a copy once they have arrived (polled, or after a stream
// synchronisation), and flag arrays are uploaded from it by DMA.  Grown by ensure(); the caller makes sure no queued work still
// uses it when it grows.
struct HostBuf {
  void* h = nullptr;  // host address
  void* d = nullptr;  // the same memory as seen by the device
  size_t bytes = 0;
  int ensure(size_t need);
  void release();
  template <class T>
  T* host() const { return reinterpret_cast<T*>(h); }
  template <class T>
  T* dev() const { return reinterpret_cast<T*>(d); }
};

}  // namespace nk
