// Host step rows with AVX2 and FMA (8 FP32 lanes); built with -mavx2 -mfma.
#include <immintrin.h>

#include "fd_cpu_rows.hpp"

namespace {

struct Avx2 {
    using V = __m256;
    static constexpr int W = 8;
    static V ld(const float *p) { return _mm256_loadu_ps(p); }
    static void st(float *p, V v) { _mm256_storeu_ps(p, v); }
    static V set1(float a) { return _mm256_set1_ps(a); }
    static V add(V a, V b) { return _mm256_add_ps(a, b); }
    static V sub(V a, V b) { return _mm256_sub_ps(a, b); }
    static V mul(V a, V b) { return _mm256_mul_ps(a, b); }
    static V fma(V a, V b, V c) { return _mm256_fmadd_ps(a, b, c); }
    static V neg(V a) { return _mm256_xor_ps(a, _mm256_set1_ps(-0.0f)); }
    // the first n lanes of v, zeros after them (0 <= n <= 8)
    static V keep(V v, int n)
    {
        const __m256i lane = _mm256_setr_epi32(0, 1, 2, 3, 4, 5, 6, 7);
        const __m256i m = _mm256_cmpgt_epi32(_mm256_set1_epi32(n), lane);
        return _mm256_and_ps(v, _mm256_castsi256_ps(m));
    }
};

}  // namespace

namespace fdcpu {

void step_rows_avx2(const Row *rows, int64_t count, int ndim)
{
    if (ndim == 3)
        for (int64_t i = 0; i < count; ++i) step_row<Avx2, 3>(rows[i]);
    else
        for (int64_t i = 0; i < count; ++i) step_row<Avx2, 2>(rows[i]);
}

}  // namespace fdcpu
