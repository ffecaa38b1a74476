// Test reference (host code only): the Philox4x32-10 words of rocRAND's
// header-only generator for the counters the method uses, to pin the
// oracle's own Philox against an independent implementation.
//
// rocRAND's philox state: key = (lo32(seed), hi32(seed)); counter words
// (x, y) = offset / 4 and (z, w) = subsequence.  With an offset of 4 (tag +
// 2^32 lo32(step)) words and subsequence = rep_id + 2^32 stream, the counter
// is (tag, lo32(step), rep_id, stream), and rocrand4() returns the 4 words of
// that counter.
#include <hip/hip_runtime.h>
#include <rocrand/rocrand_kernel.h>
#include <stdint.h>

extern "C" void rocrand_philox_words(uint64_t seed, uint32_t rep_id,
                                     uint64_t step, uint32_t stream,
                                     int64_t n, uint32_t *out) {
  for (int64_t t = 0; t < n; ++t) {
    rocrand_state_philox4x32_10 st;
    const unsigned long long sub =
        (unsigned long long)rep_id | ((unsigned long long)stream << 32);
    rocrand_init(seed, sub, 4ull * (unsigned long long)(uint32_t)t, &st);
    // counter word y = lo32(step): skip 2^32 lo32(step) counters, in four
    // skips of a quarter each (an offset counts words, four per counter)
    const unsigned long long quarter = (unsigned long long)(uint32_t)step << 32;
    for (int k = 0; k < 4; ++k) skipahead(quarter, &st);
    const uint4 w = rocrand4(&st);
    out[4 * t + 0] = w.x;
    out[4 * t + 1] = w.y;
    out[4 * t + 2] = w.z;
    out[4 * t + 3] = w.w;
  }
}
