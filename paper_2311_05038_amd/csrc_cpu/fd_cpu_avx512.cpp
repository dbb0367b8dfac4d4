// Host step rows with AVX-512F (16 FP32 lanes); built with -mavx512f.
#include <immintrin.h>

#include "fd_cpu_rows.hpp"

namespace {

struct Avx512 {
    using V = __m512;
    static constexpr int W = 16;
    static V ld(const float *p) { return _mm512_loadu_ps(p); }
    static void st(float *p, V v) { _mm512_storeu_ps(p, v); }
    static V set1(float a) { return _mm512_set1_ps(a); }
    static V add(V a, V b) { return _mm512_add_ps(a, b); }
    static V sub(V a, V b) { return _mm512_sub_ps(a, b); }
    static V mul(V a, V b) { return _mm512_mul_ps(a, b); }
    static V fma(V a, V b, V c) { return _mm512_fmadd_ps(a, b, c); }
    static V neg(V a)
    {
        return _mm512_castsi512_ps(_mm512_xor_si512(_mm512_castps_si512(a), _mm512_set1_epi32(INT32_MIN)));
    }
    static V keep(V v, int n) { return _mm512_maskz_mov_ps((__mmask16)((1u << n) - 1u), v); }
};

}  // namespace

namespace fdcpu {

void step_rows_avx512(const Row *rows, int64_t count, int ndim)
{
    if (ndim == 3)
        for (int64_t i = 0; i < count; ++i) step_row<Avx512, 3>(rows[i]);
    else
        for (int64_t i = 0; i < count; ++i) step_row<Avx512, 2>(rows[i]);
}

}  // namespace fdcpu
