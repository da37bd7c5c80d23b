// Issue-rate calibration of the vector ALU on gfx950, and a streaming read of
// known size (measurement aids; not part of the filter library's interface,
// built as libpaf_calib.so).
//
// The filter kernels are integer bit work (adds, 3-input logic, funnel
// shifts, population counts).  Whether a kernel is bound by instruction issue
// is judged against the rate at which the chip actually retires such
// instructions, so this kernel issues a known number of them and is timed
// with HIP events: every thread runs `iters` turns of a loop whose body is a
// fixed sequence of inline-asm VALU instructions over eight independent
// register chains (no memory access inside the loop; the loop counter is
// wave-uniform and lives in scalar registers).  Rate = waves x instructions
// per wave / time.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

// Instructions per loop turn of each mix (all VALU, wave64).
constexpr int kPerTurn = 16;

template <int MIX>
__device__ __forceinline__ void turn(uint32_t (&a)[8], uint32_t (&t)[8], uint32_t b, uint32_t c) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if constexpr (MIX == 0) {          // v_add_u32 only
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(a[i]) : "v"(b));
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(t[i]) : "v"(c));
        } else if constexpr (MIX == 1) {   // v_bitop3_b32 only
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0xf4" : "+v"(a[i]) : "v"(t[i]), "v"(b));
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0xde" : "+v"(t[i]) : "v"(a[i]), "v"(c));
        } else if constexpr (MIX == 2) {   // v_bcnt_u32_b32 only
            asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(a[i]) : "v"(t[i]));
            asm volatile("v_bcnt_u32_b32 %0, %1, %0" : "+v"(t[i]) : "v"(a[i]));
        } else if constexpr (MIX == 3) {   // the SneakySnake probe: add, then or-and-not
            asm volatile("v_add_u32 %0, %1, %2" : "=v"(t[i]) : "v"(a[i]), "v"(b));
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0xf4" : "+v"(a[i]) : "v"(c), "v"(t[i]));
        } else if constexpr (MIX == 4) {   // v_alignbit_b32 (funnel shift) only
            asm volatile("v_alignbit_b32 %0, %0, %1, 7" : "+v"(a[i]) : "v"(t[i]));
            asm volatile("v_alignbit_b32 %0, %0, %1, 13" : "+v"(t[i]) : "v"(a[i]));
        } else if constexpr (MIX == 5) {   // v_pk_add_u16 (two 16-bit adds) only
            asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(a[i]) : "v"(b));
            asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(t[i]) : "v"(c));
        } else if constexpr (MIX == 6) {   // map build: funnel, xor-or, nor-xor
            asm volatile("v_alignbit_b32 %0, %1, %0, 5" : "+v"(t[i]) : "v"(a[i]));
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x21" : "+v"(a[i]) : "v"(t[i]), "v"(b));
        }
    }
}

template <int MIX>
__global__ void __launch_bounds__(256) valu_kernel(uint32_t iters, uint32_t seed, uint32_t* out) {
    uint32_t a[8], t[8];
    const uint32_t x = threadIdx.x + blockIdx.x * 977u + seed;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        a[i] = x * (2u * i + 1u);
        t[i] = x ^ (0x9e3779b9u * (i + 1));
    }
    const uint32_t b = x | 1u, c = x + 12345u;
    for (uint32_t k = 0; k < iters; ++k) turn<MIX>(a, t, b, c);
    uint32_t r = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) r ^= a[i] ^ t[i];
    // Stored only for a value no input can produce, so the chains stay live
    // without any store traffic.
    if (r == 0x7fffffffu && seed == 0xffffffffu) out[0] = r;
}

const void* kernel_for(int mix) {
    switch (mix) {
        case 0: return reinterpret_cast<const void*>(&valu_kernel<0>);
        case 1: return reinterpret_cast<const void*>(&valu_kernel<1>);
        case 2: return reinterpret_cast<const void*>(&valu_kernel<2>);
        case 3: return reinterpret_cast<const void*>(&valu_kernel<3>);
        case 4: return reinterpret_cast<const void*>(&valu_kernel<4>);
        case 5: return reinterpret_cast<const void*>(&valu_kernel<5>);
        case 6: return reinterpret_cast<const void*>(&valu_kernel<6>);
        default: return nullptr;
    }
}

// Streaming read: every thread reads 16-byte vectors at a grid stride and
// folds them into one word, stored only for a value no input can produce.
__global__ void __launch_bounds__(256) read_kernel(const uint4* __restrict__ src, uint64_t n16, uint32_t seed,
                                                   uint32_t* out) {
    uint32_t r = 0;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const uint4 v = src[i];
        r ^= v.x ^ v.y ^ v.z ^ v.w;
    }
    if (r == 0x7fffffffu && seed == 0xffffffffu) out[0] = r;
}

}  // namespace

extern "C" {

// Reads n16 16-byte vectors from src [device] with `blocks` blocks of 256
// threads, `reps` times, and returns the fastest time in ms (negative on a
// HIP error).  `out` [device] is one uint32 the kernel may write.
float paf_calib_read(const void* src, uint64_t n16, uint32_t blocks, int reps, uint32_t* out) {
    if (!src || n16 == 0 || blocks == 0 || reps < 1 || !out) return -1.0f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -2.0f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -2.0f;
    }
    float best = 1e30f, rc = 0.0f;
    for (int r = 0; r <= reps && rc == 0.0f; ++r) {
        float ms = 0;
        if (hipEventRecord(e0, nullptr) != hipSuccess) rc = -3.0f;
        if (rc == 0.0f) {
            hipLaunchKernelGGL(read_kernel, dim3(blocks), dim3(256), 0, nullptr, (const uint4*)src, n16,
                               (uint32_t)r + 1u, out);
            if (hipGetLastError() != hipSuccess) rc = -3.0f;
        }
        if (rc == 0.0f && hipEventRecord(e1, nullptr) != hipSuccess) rc = -3.0f;
        if (rc == 0.0f && hipEventSynchronize(e1) != hipSuccess) rc = -4.0f;
        if (rc == 0.0f && hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -4.0f;
        if (rc == 0.0f && r > 0 && ms < best) best = ms;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc != 0.0f ? rc : best;
}

// Number of instruction mixes and the VALU instructions per loop turn.
int paf_calib_mixes(void) { return 7; }
int paf_calib_per_turn(void) { return kPerTurn; }

// Runs mix `mix` on `blocks` blocks of 256 threads for `iters` loop turns,
// `reps` times, and returns the fastest time in ms (or a negative value on a
// HIP error).  `out` [device] is one uint32 the kernel may write.
float paf_calib_valu(int mix, uint32_t blocks, uint32_t iters, int reps, uint32_t* out) {
    const void* k = kernel_for(mix);
    if (!k || blocks == 0 || reps < 1 || !out) return -1.0f;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return -2.0f;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -2.0f;
    }
    float best = 1e30f;
    uint32_t seed = 1u;
    void* args[] = {&iters, &seed, &out};
    float rc = 0.0f;
    for (int r = 0; r <= reps && rc == 0.0f; ++r) {
        seed = (uint32_t)r + 1u;
        float ms = 0;
        if (hipEventRecord(e0, nullptr) != hipSuccess) rc = -3.0f;
        else if (hipLaunchKernel(k, dim3(blocks), dim3(256), args, 0, nullptr) != hipSuccess) rc = -3.0f;
        else if (hipEventRecord(e1, nullptr) != hipSuccess) rc = -3.0f;
        else if (hipEventSynchronize(e1) != hipSuccess) rc = -4.0f;
        else if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = -4.0f;
        else if (r > 0 && ms < best) best = ms;   // turn 0 warms the clocks up
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return rc != 0.0f ? rc : best;
}

}  // extern "C"
