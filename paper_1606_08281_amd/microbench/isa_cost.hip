// isa_cost.hip -- issue cost of the VALU instructions the SSA event loop is
// made of, on gfx950.  For each instruction class a workgroup on one compute
// unit runs kIter iterations of kChains independent chains of it and reads
// the shader clock (clock64) before and after.
//   - throughput: 1024 threads, i.e. four wavefronts on each of the CU's four
//     SIMDs, all lanes active; cycles per wave64 instruction per SIMD =
//     elapsed / (4 * kIter * kChains).  The other wavefronts' loop counters
//     and branches issue beside the measured instructions, so this is the
//     SIMD's issue cost of the instruction.
//   - latency: one wavefront, one chain, minus the cycles of the same loop
//     with an empty body.
// A full-rate VALU instruction occupies its SIMD for 4 cycles (16 lanes per
// cycle): "slots" = throughput cycles / 4 is the instruction's cost in
// full-rate issue slots, the weight a lane-operation count needs.
//
// Build and run (gfx950):
//   hipcc --offload-arch=gfx950 -O3 -o isa_cost isa_cost.hip && ./isa_cost
// Prints one line per instruction class: name, throughput cycles, latency
// cycles, slots.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

constexpr int kIter = 4096;
constexpr int kChains = 8;

enum Op {
    kNone = -1,    // empty body: the loop's own cycles
    kMadU64 = 0,   // v_mad_u64_u32: 32 x 32 -> 64 multiply-add (Philox round products)
    kMulHiU32,     // v_mul_hi_u32
    kMulLoU32,     // v_mul_lo_u32
    kFmaF64,       // v_fma_f64
    kAddF64,       // v_add_f64
    kMulF64,       // v_mul_f64
    kRcpF64,       // v_rcp_f64 (the divide sequence's seed)
    kDivF64,       // a / b in binary64: IEEE-correct sequence (scale, rcp, fma refinement, fmas, fixup)
    kDivF32,       // a / b in binary32, correctly rounded
    kBitop3,       // v_bitop3_b32 (three-input bitwise operation, gfx950)
    kAddU32,       // v_add_u32
    kCvtF64U32,    // v_cvt_f64_u32
    kCmpSelF64,    // v_cmp_gt_f64 + v_cndmask_b32 (a selection step)
    kFmaF32,       // v_fma_f32 (FP32-mixed: log series, propensities)
    kCvtF32I32,    // v_cvt_f32_i32 (FP32-mixed: counts to binary32)
    kRcpF32,       // v_rcp_f32 (the binary32 divide's seed)
    kFrexpF32,     // v_frexp_mant_f32 (the binary32 log's reduction)
    kCvtF64F32,    // v_cvt_f64_f32 (FP32-mixed: the event time into the binary64 clock)
    kCndmask,      // v_cndmask_b32 alone (selections, clamps)
    kMovB32,       // v_mov_b32 (register copies the allocator leaves in the loop)
    kMovB64,       // v_mov_b64 (64-bit copies: the clock, a pair of state words)
    kCmpF64,       // v_cmp_gt_f64 into a scalar mask alone (event time against the horizon)
    kCmpU32,       // v_cmp_gt_u32 into a scalar mask (counters, bounds)
    kXorB32,       // v_xor_b32 (Philox key mixing)
    kLshrB32,      // v_lshrrev_b32 (the uniforms' mantissa bits)
    kAlignbit,     // v_alignbit_b32 (64-bit word assembly)
    kDivScaleF64,  // v_div_scale_f64 (the binary64 divide's operand scaling)
    kOps
};
static const char *kNames[kOps] = {"v_mad_u64_u32", "v_mul_hi_u32", "v_mul_lo_u32", "v_fma_f64",
                                   "v_add_f64",     "v_mul_f64",    "v_rcp_f64",    "f64 divide",
                                   "f32 divide",    "v_bitop3_b32", "v_add_u32",    "v_cvt_f64_u32",
                                   "cmp+select f64", "v_fma_f32",   "v_cvt_f32_i32", "v_rcp_f32",
                                   "v_frexp_mant_f32", "v_cvt_f64_f32", "v_cndmask_b32",
                                   "v_mov_b32",     "v_mov_b64",    "v_cmp_gt_f64", "v_cmp_gt_u32",
                                   "v_xor_b32",     "v_lshrrev_b32", "v_alignbit_b32", "v_div_scale_f64"};

template <int OP, int CH>
__device__ __forceinline__ void body(uint64_t *u, double *d, float *f, uint32_t *w,
                                     uint32_t k) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        if (OP == kMadU64) {
            uint64_t carry;
            asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0"
                         : "+v"(u[c]), "=s"(carry)
                         : "v"(w[c]), "v"(k));
        } else if (OP == kMulHiU32) {
            asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(w[c]) : "v"(k));
        } else if (OP == kMulLoU32) {
            asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(w[c]) : "v"(k));
        } else if (OP == kFmaF64) {
            asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[c]) : "v"(d[(c + 1) % CH]), "v"(d[0]));
        } else if (OP == kAddF64) {
            asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[c]) : "v"(d[(c + 1) % CH]));
        } else if (OP == kMulF64) {
            asm volatile("v_mul_f64 %0, %0, %1" : "+v"(d[c]) : "v"(d[(c + 1) % CH]));
        } else if (OP == kRcpF64) {
            asm volatile("v_rcp_f64 %0, %0" : "+v"(d[c]));
        } else if (OP == kDivF64) {
            d[c] = d[c] / d[(c + 1) % CH];
            asm volatile("" : "+v"(d[c]));
        } else if (OP == kDivF32) {
            f[c] = f[c] / f[(c + 1) % CH];
            asm volatile("" : "+v"(f[c]));
        } else if (OP == kBitop3) {
            asm volatile("v_bitop3_b32 %0, %0, %1, %2 bitop3:0x96" : "+v"(w[c]) : "v"(k), "v"(w[(c + 1) % CH]));
        } else if (OP == kAddU32) {
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(w[c]) : "v"(k));
        } else if (OP == kCvtF64U32) {
            asm volatile("v_cvt_f64_u32 %0, %1" : "=v"(d[c]) : "v"(w[c]));
            asm volatile("" : "+v"(w[c]));
        } else if (OP == kFmaF32) {
            asm volatile("v_fma_f32 %0, %0, %1, %2" : "+v"(f[c]) : "v"(f[(c + 1) % CH]), "v"(f[0]));
        } else if (OP == kCvtF32I32) {
            asm volatile("v_cvt_f32_i32 %0, %1" : "=v"(f[c]) : "v"(w[c]));
            asm volatile("" : "+v"(w[c]));
        } else if (OP == kRcpF32) {
            asm volatile("v_rcp_f32 %0, %0" : "+v"(f[c]));
        } else if (OP == kFrexpF32) {
            asm volatile("v_frexp_mant_f32 %0, %0" : "+v"(f[c]));
        } else if (OP == kCvtF64F32) {
            asm volatile("v_cvt_f64_f32 %0, %1" : "=v"(d[c]) : "v"(f[c]));
            asm volatile("" : "+v"(f[c]));
        } else if (OP == kCndmask) {
            uint64_t m = 0x5555555555555555ull;
            asm volatile("v_cndmask_b32 %0, %0, %1, %2" : "+v"(w[c]) : "v"(k), "s"(m));
        } else if (OP == kMovB32) {
            asm volatile("v_mov_b32 %0, %1" : "=v"(w[c]) : "v"(w[(c + 1) % CH]));
        } else if (OP == kMovB64) {
            asm volatile("v_mov_b64 %0, %1" : "=v"(u[c]) : "v"(u[(c + 1) % CH]));
        } else if (OP == kCmpF64) {
            uint64_t m;
            asm volatile("v_cmp_gt_f64 %0, %1, %2" : "=s"(m) : "v"(d[c]), "v"(d[(c + 1) % CH]));
            asm volatile("" ::"s"(m));
        } else if (OP == kCmpU32) {
            uint64_t m;
            asm volatile("v_cmp_gt_u32 %0, %1, %2" : "=s"(m) : "v"(w[c]), "v"(k));
            asm volatile("" ::"s"(m));
        } else if (OP == kXorB32) {
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(w[c]) : "v"(k));
        } else if (OP == kLshrB32) {
            asm volatile("v_lshrrev_b32 %0, 1, %0" : "+v"(w[c]));
        } else if (OP == kAlignbit) {
            asm volatile("v_alignbit_b32 %0, %0, %1, 7" : "+v"(w[c]) : "v"(k));
        } else if (OP == kDivScaleF64) {
            uint64_t m;
            asm volatile("v_div_scale_f64 %0, %1, %0, %2, %0" : "+v"(d[c]), "=s"(m) : "v"(d[(c + 1) % CH]));
            asm volatile("" ::"s"(m));
        } else if (OP == kCmpSelF64) {
            uint64_t m;
            asm volatile("v_cmp_gt_f64 %1, %2, %3\n\tv_cndmask_b32 %0, %0, %4, %1"
                         : "+v"(w[c]), "=s"(m)
                         : "v"(d[c]), "v"(d[(c + 1) % CH]), "v"(k));
        }
    }
}

template <int OP, int CH>
__global__ __launch_bounds__(1024) void k_cost(uint64_t *cycles, uint64_t *sink, uint32_t seed) {
    uint64_t u[CH];
    double d[CH];
    float f[CH];
    uint32_t w[CH];
    const uint32_t k = seed * 2654435761u + threadIdx.x;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
        u[c] = k + c;
        d[c] = 1.0 + 1e-3 * (double)(c + 1) + 1e-9 * (double)threadIdx.x;
        f[c] = 1.0f + 1e-3f * (float)(c + 1);
        w[c] = k ^ (0x9E3779B9u * (uint32_t)(c + 1));
    }
    // warm the instruction cache with one pass
    for (int i = 0; i < 16; ++i) body<OP, CH>(u, d, f, w, k);
    const uint64_t t0 = clock64();
    for (int i = 0; i < kIter; ++i) {
        body<OP, CH>(u, d, f, w, k);
        asm volatile("");  // the loop stays a loop (the empty-body baseline too)
    }
    const uint64_t t1 = clock64();
    uint64_t acc = 0;
#pragma unroll
    for (int c = 0; c < CH; ++c)
        acc += u[c] ^ w[c] ^ (uint64_t)__double_as_longlong(d[c]) ^ (uint64_t)__float_as_uint(f[c]);
    sink[threadIdx.x] = acc;
    __syncthreads();
    const uint64_t t2 = clock64();  // every wavefront of the workgroup is done
    if (threadIdx.x == 0) {
        cycles[0] = t1 - t0;
        cycles[1] = t2 - t0;
    }
}

// throughput: 16 wavefronts (4 per SIMD); latency: 1 wavefront, 1 chain
template <int OP>
static bool run(uint64_t *cyc, uint64_t *sink, double *thr, double *lat) {
    uint64_t h[2] = {0, 0};
    hipLaunchKernelGGL((k_cost<OP, kChains>), dim3(1), dim3(1024), 0, 0, cyc, sink, 7u);
    if (hipMemcpy(h, cyc, 16, hipMemcpyDeviceToHost) != hipSuccess) return false;
    *thr = (double)h[1] / (4.0 * kIter * kChains);
    hipLaunchKernelGGL((k_cost<OP, 1>), dim3(1), dim3(64), 0, 0, cyc, sink, 7u);
    if (hipMemcpy(h, cyc, 16, hipMemcpyDeviceToHost) != hipSuccess) return false;
    *lat = (double)h[0] / (double)kIter;
    return true;
}

int main() {
    uint64_t *cyc = nullptr, *sink = nullptr;
    if (hipMalloc(&cyc, 64) != hipSuccess || hipMalloc(&sink, 1024 * 8) != hipSuccess) {
        fprintf(stderr, "allocation failed\n");
        return 1;
    }
    double ind[kOps], dep[kOps], none_thr = 0.0, none_lat = 0.0;
    bool ok = run<kNone>(cyc, sink, &none_thr, &none_lat) && run<kMadU64>(cyc, sink, &ind[0], &dep[0]) && run<kMulHiU32>(cyc, sink, &ind[1], &dep[1]) &&
              run<kMulLoU32>(cyc, sink, &ind[2], &dep[2]) && run<kFmaF64>(cyc, sink, &ind[3], &dep[3]) &&
              run<kAddF64>(cyc, sink, &ind[4], &dep[4]) && run<kMulF64>(cyc, sink, &ind[5], &dep[5]) &&
              run<kRcpF64>(cyc, sink, &ind[6], &dep[6]) && run<kDivF64>(cyc, sink, &ind[7], &dep[7]) &&
              run<kDivF32>(cyc, sink, &ind[8], &dep[8]) && run<kBitop3>(cyc, sink, &ind[9], &dep[9]) &&
              run<kAddU32>(cyc, sink, &ind[10], &dep[10]) && run<kCvtF64U32>(cyc, sink, &ind[11], &dep[11]) &&
              run<kCmpSelF64>(cyc, sink, &ind[12], &dep[12]) && run<kFmaF32>(cyc, sink, &ind[13], &dep[13]) &&
              run<kCvtF32I32>(cyc, sink, &ind[14], &dep[14]) && run<kRcpF32>(cyc, sink, &ind[15], &dep[15]) &&
              run<kFrexpF32>(cyc, sink, &ind[16], &dep[16]) && run<kCvtF64F32>(cyc, sink, &ind[17], &dep[17]) &&
              run<kCndmask>(cyc, sink, &ind[18], &dep[18]) && run<kMovB32>(cyc, sink, &ind[19], &dep[19]) &&
              run<kMovB64>(cyc, sink, &ind[20], &dep[20]) && run<kCmpF64>(cyc, sink, &ind[21], &dep[21]) &&
              run<kCmpU32>(cyc, sink, &ind[22], &dep[22]) && run<kXorB32>(cyc, sink, &ind[23], &dep[23]) &&
              run<kLshrB32>(cyc, sink, &ind[24], &dep[24]) && run<kAlignbit>(cyc, sink, &ind[25], &dep[25]) &&
              run<kDivScaleF64>(cyc, sink, &ind[26], &dep[26]);
    if (!ok || hipDeviceSynchronize() != hipSuccess) {
        fprintf(stderr, "run failed\n");
        return 1;
    }
    printf("# empty loop: %.2f cycles per iteration (one wavefront)\n", none_lat);
    printf("%-16s %12s %12s %8s\n", "instruction", "thr_cycles", "lat_cycles", "slots");
    for (int o = 0; o < kOps; ++o)
        printf("%-16s %12.2f %12.2f %8.2f\n", kNames[o], ind[o], dep[o] - none_lat, ind[o] / 4.0);
    (void)hipFree(cyc);
    (void)hipFree(sink);
    return 0;
}
