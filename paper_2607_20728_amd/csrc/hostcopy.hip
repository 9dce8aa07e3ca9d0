// Copies between device memory and caller-owned host memory.
//
// The library never hands a pageable host pointer to the HIP runtime: every
// device <-> host transfer goes through a pinned staging buffer owned by the
// context (or network) that makes it.  The copy engine reads or writes the
// pinned pages, the calling thread copies between them and the caller's
// buffer, and the stream is synchronised before the staging buffer is
// reused.  The staging buffer grows on demand up to kStageMax bytes; larger
// transfers go in pieces of that size.
#include <algorithm>
#include <cstring>

#include "common.h"

namespace bsex {

namespace {
constexpr size_t kStageMax = (size_t)16 << 20;

int stage_reserve(HostStage* s, size_t want) {
  want = std::min(std::max(want, (size_t)4096), kStageMax);
  if (s->bytes >= want) return BSE_OK;
  if (s->p) (void)hipHostFree(s->p);
  s->p = nullptr;
  s->bytes = 0;
  size_t grow = 4096;
  while (grow < want) grow *= 2;
  grow = std::min(grow, kStageMax);
  void* p = nullptr;
  if (hipHostMalloc(&p, grow, hipHostMallocDefault) != hipSuccess || !p)
    return fail(BSE_ENOMEM, "pinned staging allocation of %zu bytes failed", grow);
  s->p = p;
  s->bytes = grow;
  return BSE_OK;
}
}  // namespace

int stage_d2h(HostStage* s, const void* dev, void* host, size_t bytes, hipStream_t st) {
  if (bytes == 0) return BSE_OK;
  if (!dev || !host) return fail(BSE_EINVAL, "device-to-host copy with a NULL pointer");
  BSE_TRY(stage_reserve(s, bytes));
  const char* d = static_cast<const char*>(dev);
  char* h = static_cast<char*>(host);
  for (size_t off = 0; off < bytes; off += s->bytes) {
    const size_t n = std::min(s->bytes, bytes - off);
    BSE_HIP(hipMemcpyAsync(s->p, d + off, n, hipMemcpyDeviceToHost, st));
    BSE_HIP(hipStreamSynchronize(st));
    std::memcpy(h + off, s->p, n);
  }
  return BSE_OK;
}

int stage_h2d(HostStage* s, const void* host, void* dev, size_t bytes, hipStream_t st) {
  if (bytes == 0) return BSE_OK;
  if (!dev || !host) return fail(BSE_EINVAL, "host-to-device copy with a NULL pointer");
  BSE_TRY(stage_reserve(s, bytes));
  const char* h = static_cast<const char*>(host);
  char* d = static_cast<char*>(dev);
  for (size_t off = 0; off < bytes; off += s->bytes) {
    const size_t n = std::min(s->bytes, bytes - off);
    // the previous piece's copy has finished (synchronised below) before
    // the staging buffer is overwritten
    std::memcpy(s->p, h + off, n);
    BSE_HIP(hipMemcpyAsync(d + off, s->p, n, hipMemcpyHostToDevice, st));
    BSE_HIP(hipStreamSynchronize(st));
  }
  return BSE_OK;
}

void stage_free(HostStage* s) {
  if (s->p) (void)hipHostFree(s->p);
  s->p = nullptr;
  s->bytes = 0;
}

}  // namespace bsex
