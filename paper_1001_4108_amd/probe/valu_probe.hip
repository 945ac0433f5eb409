// Vector-ALU issue-rate probe for gfx950 (measurement only; not part of the
// library's ABI).  Each form runs register-only loops of one instruction mix
// and reports lane-instructions per second: every thread keeps 64
// accumulators and two operand vectors of 8 values that differ per lane (read
// from memory once, so nothing folds), and the accumulators are stored at the
// end so nothing is dead.  The mixes are the inner loops of the library's
// kernels:
//   form 0  v_add_f32 alone                        (c = c + a, 64 per step)
//   form 1  fp32 min-plus, two k-steps fused       (2 v_add_f32 + 1 v_minimum3_f32
//                                                   per cell and k-pair)
//   form 2  int32 min-plus, two k-steps fused      (2 v_add_u32 + 1 v_min3_i32)
//   form 3  v_fma_f32                              (c = a * b + c)
//   form 4  bit-packed reachability                (v_and_or_b32 per word)
// and single instructions of the int32 mix, to see which part sets its rate:
//   form 5  v_add_u32 alone                        (c = c + a)
//   form 6  v_min3_i32 alone                       (c = min(c, a, b))
//   form 7  v_minimum3_f32 alone                   (c = minimum(c, a, b))
//   form 8  2 v_add_u32 + 1 v_minimum3_f32         (form 2 with the fp32
//                                                   minimum on the sums' bits)
// and the max-min semiring's loop with the two-input minima it is made of:
//   form 9  fp32 max-min, two k-steps fused        (2 two-input IEEE-2019
//                                                   minima + 1 v_maximum3_f32)
//   form 10 v_min_f32 alone                        (c = min(c, a), no operand
//                                                   quieting)
//   form 11 v_min_i32 alone                        (c = min(c, a))
// Instructions per step and thread: 192 (forms 1, 2, 8, 9), else 64.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <int FORM>
__global__ void __launch_bounds__(256) valu_kernel(const float *__restrict__ src,
                                                   float *__restrict__ dst, int iters) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    float a[8], b[8], a1[8], b1[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        a[q] = src[(t * 7 + q) & 4095];
        b[q] = src[(t * 5 + q + 8) & 4095];
        a1[q] = src[(t * 3 + q + 16) & 4095];
        b1[q] = src[(t * 11 + q + 24) & 4095];
    }
    float c[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) c[i][j] = src[(t + i * 8 + j) & 4095];
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int i = 0; i < 8; ++i)
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if constexpr (FORM == 0) {
                    c[i][j] = c[i][j] + a[i];
                } else if constexpr (FORM == 1) {
                    c[i][j] = __builtin_elementwise_minimum(
                        __builtin_elementwise_minimum(c[i][j], a[i] + b[j]), a1[i] + b1[j]);
                } else if constexpr (FORM == 2) {
                    const int x = __float_as_int(c[i][j]);
                    const int s0 = __float_as_int(a[i]) + __float_as_int(b[j]);
                    const int s1 = __float_as_int(a1[i]) + __float_as_int(b1[j]);
                    int m = x < s0 ? x : s0;
                    m = m < s1 ? m : s1;
                    c[i][j] = __int_as_float(m);
                } else if constexpr (FORM == 3) {
                    c[i][j] = __builtin_fmaf(a[i], b[j], c[i][j]);
                } else if constexpr (FORM == 5) {
                    c[i][j] = __int_as_float(__float_as_int(c[i][j]) + __float_as_int(a[i]));
                } else if constexpr (FORM == 6) {
                    const int x = __float_as_int(c[i][j]), y = __float_as_int(a[i]);
                    const int z = __float_as_int(b[j]);
                    int m = x < y ? x : y;
                    m = m < z ? m : z;
                    c[i][j] = __int_as_float(m);
                } else if constexpr (FORM == 7) {
                    c[i][j] = __builtin_elementwise_minimum(
                        __builtin_elementwise_minimum(c[i][j], a[i]), b[j]);
                } else if constexpr (FORM == 9) {
                    c[i][j] = __builtin_elementwise_maximum(
                        __builtin_elementwise_maximum(
                            c[i][j], __builtin_elementwise_minimum(a[i], b[j])),
                        __builtin_elementwise_minimum(a1[i], b1[j]));
                } else if constexpr (FORM == 10) {
                    // written out: in IEEE mode the compiler would quiet both
                    // operands first (v_max_f32 x, x, x); registers only
                    asm("v_min_f32 %0, %1, %0" : "+v"(c[i][j]) : "v"(a[i]));
                } else if constexpr (FORM == 11) {
                    const int x = __float_as_int(c[i][j]), y = __float_as_int(a[i]);
                    c[i][j] = __int_as_float(x < y ? x : y);
                } else if constexpr (FORM == 8) {
                    const int s0 = __float_as_int(a[i]) + __float_as_int(b[j]);
                    const int s1 = __float_as_int(a1[i]) + __float_as_int(b1[j]);
                    c[i][j] = __builtin_elementwise_minimum(
                        __builtin_elementwise_minimum(c[i][j], __int_as_float(s0)),
                        __int_as_float(s1));
                } else {
                    const uint32_t x = __float_as_uint(c[i][j]);
                    c[i][j] = __uint_as_float((x & __float_as_uint(a[i])) | __float_as_uint(b[j]));
                }
            }
        // operands drift so the loop body cannot be hoisted
#pragma unroll
        for (int q = 0; q < 8; ++q) asm volatile("" : "+v"(a[q]), "+v"(b[q]), "+v"(a1[q]), "+v"(b1[q]));
    }
#pragma unroll
    for (int i = 0; i < 8; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j) dst[(int64_t)t * 64 + i * 8 + j] = c[i][j];
}

}  // namespace

extern "C" {

// Instructions per loop step and thread of each form (the counts above).
int fw_probe_valu_instr_per_step(int form) {
    return (form == 1 || form == 2 || form == 8 || form == 9) ? 192 : 64;
}

// Runs `form` on `blocks` x 256 threads for `iters` steps on `stream` after
// one warm-up launch; writes the kernel time in ms (HIP events).  src: 4096
// floats of device memory; dst: blocks * 256 * 64 floats.  0 on success.
int fw_probe_valu(int form, int blocks, int iters, const float *src, float *dst, void *stream,
                  float *ms) {
    if (form < 0 || form > 11 || blocks <= 0 || iters <= 0 || !src || !dst || !ms) return 1;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return 2;
    if (hipEventCreate(&e1) != hipSuccess) return 2;
    auto go = [&](int n) {
        switch (form) {
        case 0: valu_kernel<0><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 1: valu_kernel<1><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 2: valu_kernel<2><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 3: valu_kernel<3><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 4: valu_kernel<4><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 5: valu_kernel<5><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 6: valu_kernel<6><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 7: valu_kernel<7><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 8: valu_kernel<8><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 9: valu_kernel<9><<<blocks, 256, 0, st>>>(src, dst, n); break;
        case 10: valu_kernel<10><<<blocks, 256, 0, st>>>(src, dst, n); break;
        default: valu_kernel<11><<<blocks, 256, 0, st>>>(src, dst, n); break;
        }
    };
    go(iters);
    int rc = hipEventRecord(e0, st) == hipSuccess ? 0 : 2;
    go(iters);
    if (hipEventRecord(e1, st) != hipSuccess) rc = 2;
    if (hipGetLastError() != hipSuccess) rc = 2;
    if (hipEventSynchronize(e1) != hipSuccess) rc = 2;
    if (rc == 0 && hipEventElapsedTime(ms, e0, e1) != hipSuccess) rc = 2;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc;
}

}  // extern "C"
