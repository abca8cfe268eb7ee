// Debug controls of the library (failure tests).
#include <atomic>

#include "ctx.h"
#include "../../include/mbw.h"

std::atomic<unsigned long long> g_mbw_mem_limit{0};

extern "C" int mbw_debug_set_mem_limit(uint64_t bytes) {
  g_mbw_mem_limit.store(bytes, std::memory_order_relaxed);
  return MBW_OK;
}
