// Sorting and scan primitives used by the index bookkeeping (rocPRIM).
#include <cstring>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "common.h"

namespace hif {

namespace {
void* temp(DBuf<unsigned char>& scratch, size_t bytes, MemTracker* mt) {
  scratch.ensure(bytes ? bytes : 1, mt);
  return scratch.p;
}
}  // namespace

void sort_u64(uint64_t* keys, uint64_t* tmp, size_t n, int end_bit, hipStream_t s,
              DBuf<unsigned char>& scratch, MemTracker* mt) {
  if (n <= 1) return;
  size_t bytes = 0;
  HIF_HIP(rocprim::radix_sort_keys(nullptr, bytes, keys, tmp, n, 0, end_bit, s));
  void* t = temp(scratch, bytes, mt);
  HIF_HIP(rocprim::radix_sort_keys(t, bytes, keys, tmp, n, 0, end_bit, s));
  HIF_HIP(hipMemcpyAsync(keys, tmp, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
}

void sort_u64_i32(uint64_t* keys, uint64_t* ktmp, int32_t* vals, int32_t* vtmp, size_t n,
                  int end_bit, hipStream_t s, DBuf<unsigned char>& scratch, MemTracker* mt) {
  if (n <= 1) return;
  size_t bytes = 0;
  HIF_HIP(rocprim::radix_sort_pairs(nullptr, bytes, keys, ktmp, vals, vtmp, n, 0, end_bit, s));
  void* t = temp(scratch, bytes, mt);
  HIF_HIP(rocprim::radix_sort_pairs(t, bytes, keys, ktmp, vals, vtmp, n, 0, end_bit, s));
  HIF_HIP(hipMemcpyAsync(keys, ktmp, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
  HIF_HIP(hipMemcpyAsync(vals, vtmp, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
}

void sort_i32_i32(int32_t* keys, int32_t* ktmp, int32_t* vals, int32_t* vtmp, size_t n,
                  int end_bit, hipStream_t s, DBuf<unsigned char>& scratch, MemTracker* mt) {
  if (n <= 1) return;
  size_t bytes = 0;
  HIF_HIP(rocprim::radix_sort_pairs(nullptr, bytes, keys, ktmp, vals, vtmp, n, 0, end_bit, s));
  void* t = temp(scratch, bytes, mt);
  HIF_HIP(rocprim::radix_sort_pairs(t, bytes, keys, ktmp, vals, vtmp, n, 0, end_bit, s));
  HIF_HIP(hipMemcpyAsync(keys, ktmp, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  HIF_HIP(hipMemcpyAsync(vals, vtmp, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
}

void exclusive_scan_i64(const int64_t* in, int64_t* out, size_t n, hipStream_t s,
                        DBuf<unsigned char>& scratch, MemTracker* mt) {
  // out[0..n]: out[n] = total.  Scan n+1 items where the last input reads as 0
  // is avoided by scanning n items and adding the tail separately.
  if (n == 0) {
    HIF_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
    return;
  }
  size_t bytes = 0;
  HIF_HIP(rocprim::inclusive_scan(nullptr, bytes, in, out + 1, n, rocprim::plus<int64_t>(), s));
  void* t = temp(scratch, bytes, mt);
  HIF_HIP(rocprim::inclusive_scan(t, bytes, in, out + 1, n, rocprim::plus<int64_t>(), s));
  HIF_HIP(hipMemsetAsync(out, 0, sizeof(int64_t), s));
}

void exclusive_scan_i32(const int32_t* in, int32_t* out, size_t n, hipStream_t s,
                        DBuf<unsigned char>& scratch, MemTracker* mt) {
  if (n == 0) {
    HIF_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
    return;
  }
  size_t bytes = 0;
  HIF_HIP(rocprim::inclusive_scan(nullptr, bytes, in, out + 1, n, rocprim::plus<int32_t>(), s));
  void* t = temp(scratch, bytes, mt);
  HIF_HIP(rocprim::inclusive_scan(t, bytes, in, out + 1, n, rocprim::plus<int32_t>(), s));
  HIF_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
}

}  // namespace hif
