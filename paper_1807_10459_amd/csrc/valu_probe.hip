// VALU throughput probe: the issue rate of the instruction classes the search kernels use,
// measured on the running device, so that the roofline peak is a measurement of this part
// rather than a datasheet reading.  Each lane runs 16 independent chains of one instruction
// class; no memory traffic inside the timed loop.
#include <hip/hip_runtime.h>

#include "../../include/ksgcmi.h"
#include "runtime.h"

namespace ksg {

template <int KIND>
__global__ __launch_bounds__(256) void valu_probe_kernel(int iters, float seed, float* __restrict__ out) {
  float a[16];
  unsigned c[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    a[i] = seed + (float)(threadIdx.x + i);
    c[i] = threadIdx.x + i;
  }
  const float s = seed * 0.5f;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      if constexpr (KIND == 0) {  // FP32 subtract (VOP2)
        asm volatile("v_sub_f32 %0, %0, %1" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 1) {  // FP32 max3 with |.| modifiers (VOP3)
        asm volatile("v_max3_f32 %0, |%0|, |%1|, %0" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 2) {  // FP32 compare to VCC + add-with-carry count (VOPC + VOP2)
        asm volatile("v_cmp_lt_f32 vcc, %1, %2\n\tv_addc_co_u32 %0, vcc, 0, %0, vcc"
                     : "+v"(c[i]) : "v"(a[i]), "v"(s) : "vcc");
      } else if constexpr (KIND == 3) {  // FP32 median of three (VOP3)
        asm volatile("v_med3_f32 %0, %0, %1, %0" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 4) {  // FP32 fused multiply-add (VOP3)
        asm volatile("v_fma_f32 %0, %0, %1, %1" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 5) {  // FP32 max (VOP2, no modifiers)
        asm volatile("v_max_f32 %0, %0, %1" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 6) {  // FP32 max with |.| (VOP3 encoding)
        asm volatile("v_max_f32_e64 %0, |%0|, %1" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 7) {  // u32 min (VOP2)
        asm volatile("v_min_u32 %0, %0, %1" : "+v"(c[i]) : "v"(c[0]));
      } else if constexpr (KIND == 8) {  // select by VCC (VOP2)
        asm volatile("v_cndmask_b32 %0, %0, %1, vcc" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 9) {  // u32 add (VOP2)
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(c[i]) : "v"(c[0]));
      } else if constexpr (KIND == 10) {  // FP32 compare into an SGPR pair (VOP3)
        asm volatile("v_cmp_lt_f32_e64 s[40:41], %0, %1" : : "v"(a[i]), "v"(s) : "s40", "s41");
      } else if constexpr (KIND == 11) {  // bitwise and (VOP2)
        asm volatile("v_and_b32 %0, %0, %1" : "+v"(c[i]) : "v"(c[0]));
      } else if constexpr (KIND == 12) {  // FP32 subtract with an SGPR operand (VOP2)
        asm volatile("v_sub_f32 %0, %1, %0" : "+v"(a[i]) : "s"(seed));
      } else if constexpr (KIND == 13) {  // FP32 min3 (VOP3)
        asm volatile("v_min3_f32 %0, %0, %1, %0" : "+v"(a[i]) : "v"(s));
      } else if constexpr (KIND == 14) {  // u32 subtract (VOP2)
        asm volatile("v_sub_u32 %0, %0, %1" : "+v"(c[i]) : "v"(c[0]));
      } else if constexpr (KIND == 15) {  // logical shift right (VOP2)
        asm volatile("v_lshrrev_b32 %0, 1, %0" : "+v"(c[i]));
      } else if constexpr (KIND == 16) {  // u32 add of three operands (VOP3)
        asm volatile("v_add3_u32 %0, %0, %1, %0" : "+v"(c[i]) : "v"(c[0]));
      } else {  // move from an SGPR (VOP1)
        asm volatile("v_mov_b32 %0, %1" : "=v"(a[i]) : "s"(seed + (float)i));
      }
    }
  }
  float acc = 0.0f;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc += a[i] + (float)c[i];
  if (acc == 12345.678f) out[threadIdx.x] = acc;  // keeps the chains live
}

// LDS read bandwidth: each lane reads 8 independent float4 values per iteration from a 64 KB
// LDS array (consecutive lanes at consecutive 16-byte addresses, so no bank conflicts), the
// address alternating between its two halves so that the reads cannot be hoisted out of the
// loop; all 8 reads are issued before empty asm statements take the loaded registers, so the
// reads stay 128-bit, overlap, and no arithmetic follows them.
__global__ __launch_bounds__(256) void lds_probe_kernel(int iters, float seed, float* __restrict__ out) {
  constexpr int kHalf = 2048;  // float4 per half
  __shared__ float4 s[2 * kHalf];
  for (int i = (int)threadIdx.x; i < 2 * kHalf; i += 256)
    s[i] = make_float4(seed + (float)i, seed - (float)i, seed * (float)i, (float)i);
  __syncthreads();
  const int lane = (int)threadIdx.x;
  for (int it = 0; it < iters; ++it) {
    const float4* h = s + (it & 1) * kHalf + lane;
    float4 v[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = h[i * 256];  // all 8 reads in flight before the first use
#pragma unroll
    for (int i = 0; i < 8; ++i) asm volatile("" : : "v"(v[i].x), "v"(v[i].y), "v"(v[i].z), "v"(v[i].w));
  }
  if (seed == 12345.678f) out[threadIdx.x] = s[lane].x;
}

}  // namespace ksg

using namespace ksg;

extern "C" int ksg_lds_probe(ksg_ctx* c, int32_t iters, double* bytes_per_s) {
  if (!c) return KSG_EINVAL;
  if (!bytes_per_s || iters < 1) return c->fail(KSG_EINVAL, "ksg_lds_probe: bad argument");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(KSG_EDEVICE, "hipSetDevice");
  const int blocks = c->cus * 8;
  int st = c->reserve(c->tmp, 256 * sizeof(float), "probe output");
  if (st) return st;
  float seed = 1.25f;
  float* out = (float*)c->tmp.ptr;
  void* args[] = {&iters, &seed, &out};
  hipEvent_t e0 = c->get_event(), e1 = c->get_event();
  if (!e0 || !e1) return c->fail(KSG_EDEVICE, "events");
  const void* fn = (const void*)&lds_probe_kernel;
  hipError_t e = hipLaunchKernel(fn, dim3(blocks), dim3(256), args, 0, c->stream);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  if (e == hipSuccess) e = hipLaunchKernel(fn, dim3(blocks), dim3(256), args, 0, c->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  c->event_pool.push_back(e0);
  c->event_pool.push_back(e1);
  if (e != hipSuccess) return c->hip_fail(e, "lds probe");
  *bytes_per_s = (double)iters * 8.0 * 16.0 * 256.0 * (double)blocks / (ms * 1e-3);
  return KSG_OK;
}

extern "C" int ksg_valu_probe(ksg_ctx* c, int32_t kind, int32_t iters, double* lane_ops_per_s) {
  if (!c) return KSG_EINVAL;
  if (!lane_ops_per_s || kind < 0 || kind > 17 || iters < 1) return c->fail(KSG_EINVAL, "ksg_valu_probe: bad argument");
  if (hipSetDevice(c->device) != hipSuccess) return c->fail(KSG_EDEVICE, "hipSetDevice");
  const void* fns[18] = {(const void*)&valu_probe_kernel<0>,  (const void*)&valu_probe_kernel<1>,
                         (const void*)&valu_probe_kernel<2>,  (const void*)&valu_probe_kernel<3>,
                         (const void*)&valu_probe_kernel<4>,  (const void*)&valu_probe_kernel<5>,
                         (const void*)&valu_probe_kernel<6>,  (const void*)&valu_probe_kernel<7>,
                         (const void*)&valu_probe_kernel<8>,  (const void*)&valu_probe_kernel<9>,
                         (const void*)&valu_probe_kernel<10>, (const void*)&valu_probe_kernel<11>,
                         (const void*)&valu_probe_kernel<12>, (const void*)&valu_probe_kernel<13>,
                         (const void*)&valu_probe_kernel<14>, (const void*)&valu_probe_kernel<15>,
                         (const void*)&valu_probe_kernel<16>, (const void*)&valu_probe_kernel<17>};
  const int blocks = c->cus * 16;
  int st = c->reserve(c->tmp, 256 * sizeof(float), "probe output");
  if (st) return st;
  float seed = 1.25f;
  float* out = (float*)c->tmp.ptr;
  void* args[] = {&iters, &seed, &out};
  hipEvent_t e0 = c->get_event(), e1 = c->get_event();
  if (!e0 || !e1) return c->fail(KSG_EDEVICE, "events");
  hipError_t e = hipLaunchKernel(fns[kind], dim3(blocks), dim3(256), args, 0, c->stream);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, c->stream);
  if (e == hipSuccess) e = hipLaunchKernel(fns[kind], dim3(blocks), dim3(256), args, 0, c->stream);
  if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  c->event_pool.push_back(e0);
  c->event_pool.push_back(e1);
  if (e != hipSuccess) return c->hip_fail(e, "valu probe");
  const double per_lane = (double)iters * 16.0 * (kind == 2 ? 2.0 : 1.0);
  *lane_ops_per_s = per_lane * 256.0 * (double)blocks / (ms * 1e-3);
  return KSG_OK;
}
