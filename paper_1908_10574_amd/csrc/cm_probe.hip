// cm_probe.hip -- measured VALU peak rates of the instructions the
// Smith-Waterman cell update is made of (the denominators of its roofline).
//
// Every thread runs 32 independent dependency chains of one instruction,
// written in inline asm so that each source operation is exactly one VALU
// instruction (no loads or stores inside the loop).  The grid holds 8 blocks
// of 256 threads per compute unit (8 wavefronts per SIMD).  Thread 0 of block
// 0 reads the shader cycle counter and the constant-rate real-time counter
// around its loop, which gives the clock the chip ran at.
#include "../../include/cm.h"
#include "cm_runtime.h"

namespace {

constexpr int kChains = 32;

template <int KIND>
__global__ __launch_bounds__(256) void k_valu_probe(uint32_t* out, int iters, unsigned long long* clk) {
    uint32_t v[kChains];
#pragma unroll
    for (int k = 0; k < kChains; ++k) v[k] = threadIdx.x * 0x00010001u + k;
    const uint32_t b = (blockIdx.x & 7) * 0x00010001u + 1u, c = 0x00030003u;
    unsigned long long c0 = 0, r0 = 0;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        c0 = clock64();
        r0 = wall_clock64();
    }
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kChains; ++k) {
            if constexpr (KIND == CM_PROBE_I32_ADD) {
                asm volatile("v_add_u32 %0, %0, %1" : "+v"(v[k]) : "v"(b));
            } else if constexpr (KIND == CM_PROBE_I32_MAX3) {
                asm volatile("v_max3_i32 %0, %0, %1, %2" : "+v"(v[k]) : "v"(b), "v"(c));
            } else if constexpr (KIND == CM_PROBE_PK16_ADD) {
                asm volatile("v_pk_add_u16 %0, %0, %1" : "+v"(v[k]) : "v"(b));
            } else {
                asm volatile("v_pk_maximum3_f16 %0, %0, %1, %2" : "+v"(v[k]) : "v"(b), "v"(c));
            }
        }
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kChains; ++k) acc ^= v[k];
    out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        clk[0] = clock64() - c0;
        clk[1] = wall_clock64() - r0;
    }
}

}  // namespace

extern "C" cm_status cm_probe_valu(cm_context* ctx, int kind, double* ops_per_second, double* clock_hz) {
    CM_TRY
    if (!ctx || !ops_per_second || kind < CM_PROBE_I32_ADD || kind > CM_PROBE_PK16_MAX3)
        return cmrt::fail(CM_EINVAL, "bad argument");
    hipError_t e = hipSetDevice(ctx->device);
    if (e != hipSuccess) return cmrt::hip_fail(e, "hipSetDevice");
    const int blocks = ctx->n_cu * 8, threads = 256, iters = 100000;
    const size_t out_bytes = static_cast<size_t>(blocks) * threads * 4;
    cmrt::DeviceBuf& buf = ctx->drv[2];   // not used by the driver
    if (!buf.ensure(out_bytes + 64)) return cmrt::fail(CM_ENOMEM, "probe output");
    uint32_t* out = static_cast<uint32_t*>(buf.ptr);
    unsigned long long* clk = reinterpret_cast<unsigned long long*>(static_cast<char*>(buf.ptr) + out_bytes);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if ((e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return cmrt::hip_fail(e, "events");
    }
    auto launch = [&](int n_iter) {
        switch (kind) {
            case CM_PROBE_I32_ADD:
                hipLaunchKernelGGL(k_valu_probe<CM_PROBE_I32_ADD>, dim3(blocks), dim3(threads), 0, nullptr, out, n_iter, clk);
                break;
            case CM_PROBE_I32_MAX3:
                hipLaunchKernelGGL(k_valu_probe<CM_PROBE_I32_MAX3>, dim3(blocks), dim3(threads), 0, nullptr, out, n_iter, clk);
                break;
            case CM_PROBE_PK16_ADD:
                hipLaunchKernelGGL(k_valu_probe<CM_PROBE_PK16_ADD>, dim3(blocks), dim3(threads), 0, nullptr, out, n_iter, clk);
                break;
            default:
                hipLaunchKernelGGL(k_valu_probe<CM_PROBE_PK16_MAX3>, dim3(blocks), dim3(threads), 0, nullptr, out, n_iter, clk);
                break;
        }
    };
    launch(iters / 10);   // warm-up (clocks ramp up)
    (void)hipEventRecord(e0, nullptr);
    launch(iters);
    (void)hipEventRecord(e1, nullptr);
    e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    unsigned long long h_clk[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpy(h_clk, clk, sizeof(h_clk), hipMemcpyDeviceToHost);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return cmrt::hip_fail(e, "probe");
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || wall_khz <= 0)
        wall_khz = 100000;   // the documented 100 MHz real-time counter
    const double lanes = static_cast<double>(blocks) * threads * iters * kChains;
    const double per_lane = (kind == CM_PROBE_PK16_ADD || kind == CM_PROBE_PK16_MAX3) ? 2.0 : 1.0;
    *ops_per_second = lanes * per_lane / (ms * 1e-3);
    if (clock_hz)
        *clock_hz = h_clk[1] ? static_cast<double>(h_clk[0]) / (static_cast<double>(h_clk[1]) / (wall_khz * 1e3)) : 0.0;
    return CM_OK;
    CM_CATCH
}
