// Stable key/value sort and integer prefix sum used to bin constraint rows by
// lattice cell (rocPRIM, header-only).  Both are deterministic: the radix sort
// is stable and integer sums are exact.
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "vd_kernels.h"

namespace vd {

size_t sort_temp_bytes(int n) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs(nullptr, bytes, (const unsigned*)nullptr, (unsigned*)nullptr,
                            (const int*)nullptr, (int*)nullptr, n, 0u, 32u);
  return bytes;
}

hipError_t sort_pairs(void* temp, size_t bytes, const unsigned* kin, unsigned* kout,
                      const int* vin, int* vout, int n, int end_bit, hipStream_t s) {
  if (n == 0) return hipSuccess;
  return rocprim::radix_sort_pairs(temp, bytes, kin, kout, vin, vout, n, 0u,
                                   (unsigned)end_bit, s);
}

size_t scan_temp_bytes(int n) {
  size_t bytes = 0;
  (void)rocprim::exclusive_scan(nullptr, bytes, (const int*)nullptr, (int*)nullptr, 0, (size_t)n,
                          rocprim::plus<int>());
  return bytes;
}

hipError_t exclusive_scan(void* temp, size_t bytes, const int* in, int* out, int n,
                          hipStream_t s) {
  if (n == 0) return hipSuccess;
  return rocprim::exclusive_scan(temp, bytes, in, out, 0, (size_t)n, rocprim::plus<int>(), s);
}

}  // namespace vd
