// Streaming-bandwidth probe for the roofline context of the TV sweep (built into
// lib/libeptv_probe.so, separate from the EP library; only the benchmark loads it).
//
// The sweep reads five site planes and writes four (each site one float2 per
// pixel).  The probe moves the same nine planes with the same accesses and no
// arithmetic beyond one add per word, so its rate is what this access pattern
// can reach on the device: the practical ceiling the sweep's fraction of peak is
// read against.
//   mode 0: flat, one 16-byte word (two pixels) of every plane per thread;
//   mode 1: marching like the sweep, one wave per 128-column strip and a chunk
//           of `chunk_rows` rows, four waves per block on consecutive chunks,
//           one row per iteration.
// Every access stays inside rows [0, h) x columns [0, w) of planes with row
// pitch w; w must be a multiple of 128 (mode 1) or 2 (mode 0).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

struct Planes {
  const float4* in[5];
  float4* out[4];
};

__device__ __forceinline__ void move_word(const Planes& p, long long i) {
  const float4 a = p.in[0][i], b = p.in[1][i], c = p.in[2][i], d = p.in[3][i], e = p.in[4][i];
  p.out[0][i] = make_float4(a.x + e.x, a.y, a.z, a.w);
  p.out[1][i] = make_float4(b.x + e.y, b.y, b.z, b.w);
  p.out[2][i] = make_float4(c.x + e.z, c.y, c.z, c.w);
  p.out[3][i] = make_float4(d.x + e.w, d.y, d.z, d.w);
}

__global__ __launch_bounds__(256) void k_stream_flat(Planes p, long long words) {
  const long long i = (long long)blockIdx.x * 256 + threadIdx.x;
  if (i < words) move_word(p, i);
}

__global__ __launch_bounds__(256) void k_stream_march(Planes p, int h, int w, int chunk_rows) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int strips = w / 128;
  const int chunk = blockIdx.x / strips * 4 + wave;
  const int strip = blockIdx.x % strips;
  const int r0 = chunk * chunk_rows;
  const int r1 = min(r0 + chunk_rows, h);
  for (int r = r0; r < r1; ++r) move_word(p, ((long long)r * w + strip * 128) / 2 + lane);
}

}  // namespace

// One launch of the probe on `stream` over planes in[0..4] (read) and out[0..3]
// (written), each h x w float2 (device pointers, 16-byte aligned).  Returns 0, or
// -1 for bad arguments, or the HIP error code of the launch.
extern "C" int eptv_stream_probe(const void* const* in, void* const* out, int h, int w, int mode,
                                 int chunk_rows, void* stream) {
  if (!in || !out || h <= 0 || w <= 0 || (mode != 0 && mode != 1)) return -1;
  if (mode == 0 && w % 2 != 0) return -1;
  if (mode == 1 && (w % 128 != 0 || chunk_rows <= 0)) return -1;
  Planes p;
  for (int k = 0; k < 5; ++k) {
    if (!in[k]) return -1;
    p.in[k] = static_cast<const float4*>(in[k]);
  }
  for (int k = 0; k < 4; ++k) {
    if (!out[k]) return -1;
    p.out[k] = static_cast<float4*>(out[k]);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long words = (long long)h * w / 2;
  if (mode == 0) {
    hipLaunchKernelGGL(k_stream_flat, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s, p,
                       words);
  } else {
    const int chunks = (h + chunk_rows - 1) / chunk_rows;
    const int blocks = (chunks + 3) / 4 * (w / 128);
    hipLaunchKernelGGL(k_stream_march, dim3(blocks), dim3(256), 0, s, p, h, w, chunk_rows);
  }
  const hipError_t e = hipGetLastError();
  return e == hipSuccess ? 0 : (int)e;
}
