// Issue-rate probes: float32 VOP2/VOP3 arithmetic, the hardware reciprocal, the direct sum's
// per-pair instruction mix and the FP64 add, each issued as 16 independent register chains per
// lane at full occupancy.  The instructions are written as inline assembly (register operands
// only, no memory access) so the compiler neither removes nor reshapes them.
#include "rs_internal.h"
#include "rs_probe.h"

namespace rs {

namespace {

constexpr int kChains = 16;

template <int OP>
__global__ void __launch_bounds__(256) k_probe(int iters, float seed)
{
    float r[kChains];
#pragma unroll
    for (int i = 0; i < kChains; ++i) r[i] = seed + (float)(threadIdx.x + 3 * i + 1);
    double d[kChains / 2];
#pragma unroll
    for (int i = 0; i < kChains / 2; ++i) d[i] = (double)r[i];
    const float a = 0.999999f, b = 1.0e-7f;
    const double e = 1.0e-300;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int rep = 0; rep < 8; ++rep) {
#pragma unroll
            for (int i = 0; i < kChains; ++i) {
                if constexpr (OP == RS_PROBE_FMAC_F32) {
                    asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(r[i]) : "v"(a), "v"(b));
                } else if constexpr (OP == RS_PROBE_FMA_F32) {
                    asm volatile("v_fma_f32 %0, %1, %0, %2" : "+v"(r[i]) : "v"(a), "v"(b));
                } else if constexpr (OP == RS_PROBE_MUL_F32) {
                    asm volatile("v_mul_f32 %0, %1, %0" : "+v"(r[i]) : "v"(a));
                } else if constexpr (OP == RS_PROBE_RCP_F32) {
                    asm volatile("v_rcp_f32 %0, %0" : "+v"(r[i]));
                } else if constexpr (OP == RS_PROBE_MIX_13_1) {
                    // chains 0-12 take an FMA, chain 13 a reciprocal: 13 : 1 per 14 instructions
                    if (i < 13) asm volatile("v_fmac_f32 %0, %1, %2" : "+v"(r[i]) : "v"(a), "v"(b));
                    else if (i == 13) asm volatile("v_rcp_f32 %0, %0" : "+v"(r[i]));
                } else if constexpr (OP == RS_PROBE_ADD_F64) {
                    if (i < kChains / 2) asm volatile("v_add_f64 %0, %0, %1" : "+v"(d[i]) : "v"(e));
                }
            }
        }
    }
    // keep the chains live (never true for the seeds used: the values stay finite)
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < kChains; ++i) acc += r[i];
#pragma unroll
    for (int i = 0; i < kChains / 2; ++i) acc += (float)d[i];
    if (acc == 1234.5f) asm volatile("s_nop 0");
}

template <int OP>
hipError_t probe_launch(int blocks, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(k_probe<OP>, dim3((unsigned)blocks), dim3(256), 0, s, iters, 1.0f);
    return hipGetLastError();
}

}  // namespace

int probe_ops_per_iter(int op)
{
    switch (op) {
    case RS_PROBE_MIX_13_1: return 8 * 14;
    case RS_PROBE_ADD_F64: return 8 * (kChains / 2);
    default: return 8 * kChains;
    }
}

hipError_t launch_probe(int op, int blocks, int iters, hipStream_t s)
{
    switch (op) {
    case RS_PROBE_FMAC_F32: return probe_launch<RS_PROBE_FMAC_F32>(blocks, iters, s);
    case RS_PROBE_FMA_F32: return probe_launch<RS_PROBE_FMA_F32>(blocks, iters, s);
    case RS_PROBE_MUL_F32: return probe_launch<RS_PROBE_MUL_F32>(blocks, iters, s);
    case RS_PROBE_RCP_F32: return probe_launch<RS_PROBE_RCP_F32>(blocks, iters, s);
    case RS_PROBE_MIX_13_1: return probe_launch<RS_PROBE_MIX_13_1>(blocks, iters, s);
    case RS_PROBE_ADD_F64: return probe_launch<RS_PROBE_ADD_F64>(blocks, iters, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace rs
