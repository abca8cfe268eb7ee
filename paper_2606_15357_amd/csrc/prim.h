// Device-wide sorts, scans and selections of the glue steps (everything but the hot kernels), on
// rocPRIM.  Each call follows the usual two-phase protocol: with tmp == nullptr it only writes the
// temporary storage it needs to `bytes`.
#pragma once
#include <cstring>   // before rocPRIM: its headers use memset in host code
#include <iterator>
#include <utility>

#include <rocprim/rocprim.hpp>

namespace prim {

template <class T>
using dbuf = rocprim::double_buffer<T>;

// out[i] = in[0] + ... + in[i-1], out[0] = 0; summed in the type a sum of two inputs has
template <class I, class O>
inline hipError_t exclusive_sum(void *tmp, size_t &bytes, I in, O out, size_t n, hipStream_t st) {
  using T = typename std::iterator_traits<I>::value_type;
  using A = decltype(std::declval<T>() + std::declval<T>());
  return rocprim::exclusive_scan(tmp, bytes, in, out, A(0), n, rocprim::plus<A>(), st);
}

// out[i] = max(in[0], ..., in[i])
template <class I, class O>
inline hipError_t inclusive_max(void *tmp, size_t &bytes, I in, O out, size_t n, hipStream_t st) {
  using T = typename std::iterator_traits<I>::value_type;
  return rocprim::inclusive_scan(tmp, bytes, in, out, n, rocprim::maximum<T>(), st);
}

// stable LSD radix sort of (key, value) pairs on key bits [b0, b1); k.current() / v.current() hold
// the result afterwards
template <class K, class V>
inline hipError_t sort_pairs(void *tmp, size_t &bytes, dbuf<K> &k, dbuf<V> &v, size_t n, int b0, int b1,
                             hipStream_t st) {
  return rocprim::radix_sort_pairs(tmp, bytes, k, v, n, (unsigned)b0, (unsigned)b1, st);
}

// the same sort through rocPRIM's merge-based path at every size.  Above 2^20 items the default
// dispatch takes the onesweep path, which resets its histogram and look-back states with
// hipMemsetAsync; a captured graph must not record memset operations (they are not reliable when
// the graph is replayed), and the merge-based path issues none.
template <class K, class V>
inline hipError_t sort_pairs_merge(void *tmp, size_t &bytes, dbuf<K> &k, dbuf<V> &v, size_t n, int b0, int b1,
                                   hipStream_t st) {
  using cfg = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config, rocprim::default_config,
                                         ~size_t(0)>;
  return rocprim::radix_sort_pairs<cfg>(tmp, bytes, k, v, n, (unsigned)b0, (unsigned)b1, st);
}

// the indices i < n with flags[i] != 0, ascending, into out; their number into *count (device)
template <class F, class O, class C>
inline hipError_t flagged_indices(void *tmp, size_t &bytes, F flags, O out, C count, size_t n, hipStream_t st) {
  return rocprim::select(tmp, bytes, rocprim::counting_iterator<uint32_t>(0), flags, out, count, n, st);
}

}  // namespace prim
