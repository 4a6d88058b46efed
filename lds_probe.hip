// LDS access-pattern probe for the step kernel's bank-conflict counters.
// Each kernel repeats one LDS access pattern of the fused step kernel (or a
// plain linear reference) on a 152 KB LDS array, so that
//   rocprofv3 --pmc SQ_LDS_BANK_CONFLICT SQ_LDS_IDX_ACTIVE -- ./lds_probe
// gives the counters of each pattern alone.  Strides of the two working-size
// workloads: 3D 8x128 (S = 132, S2 = 132, 128 columns, Wp = 128) and 2D 8x100
// (S = 132, S2 = 100, 96 columns, Wp = 112).  Build: hipcc --offload-arch=gfx950
// -O3 -Xclang -target-feature -Xclang -packed-fp32-ops lds_probe.hip -o
// lds_probe.  Not part of the library.
#include <hip/hip_runtime.h>
#include <cstdio>
typedef float v4f __attribute__((ext_vector_type(4)));
constexpr int REP = 64;
// params: S (stride of [col][neuron]), S2 (stride of [neuron][col]), NCOL
struct P { int S, S2, NCOL, Wp, KC; };

// forward B read: bb = buf + j*S + g*4*KC + cb*16*S + 4*s4
__global__ __launch_bounds__(512) void k_fwdB(P p, float* out) {
  extern __shared__ float lds[];
  for (int i = threadIdx.x; i < 38000; i += blockDim.x) lds[i] = i;
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  v4f acc = {0, 0, 0, 0};
  for (int r = 0; r < REP; ++r)
    for (int cb = 0; cb < p.NCOL / 16; ++cb)
      for (int s4 = 0; s4 < p.KC; ++s4)
        acc += *reinterpret_cast<const v4f*>(lds + j * p.S + g * 4 * p.KC + cb * 16 * p.S + 4 * s4);
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc[0] + acc[1] + acc[2] + acc[3];
}
// store_fwd: buf + (16*cb + j)*S + 16*w + 4*g  (b128 write)
__global__ __launch_bounds__(512) void k_storefwd(P p, float* out) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  v4f v = {1.f * lane, 2, 3, 4};
  for (int r = 0; r < REP; ++r)
    for (int cb = 0; cb < p.NCOL / 16; ++cb) {
      *reinterpret_cast<v4f*>(lds + (16 * cb + j) * p.S + 16 * w + 4 * g) = v;
      v[1] += 1.f;
    }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = lds[threadIdx.x];
}
// act_store_bwd: row = buf + (16w + 4g + i)*S2 + j; row[16*cb]  (b32 write)
__global__ __launch_bounds__(512) void k_actbwd(P p, float* out) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  float v = lane;
  for (int r = 0; r < REP; ++r)
    for (int i = 0; i < 4; ++i)
      for (int cb = 0; cb < p.NCOL / 16; ++cb) {
        lds[(16 * w + 4 * g + i) * p.S2 + j + 16 * cb] = v;
        v += 1.f;
      }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = lds[threadIdx.x];
}
// gemm_dw A read: ab = buf + 4g*S + 16w + j; ab[(16*s4+q)*S]  (b32 read)
__global__ __launch_bounds__(512) void k_dwA(P p, float* out) {
  extern __shared__ float lds[];
  for (int i = threadIdx.x; i < 38000; i += blockDim.x) lds[i] = i;
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  float acc = 0;
  for (int r = 0; r < REP; ++r)
    for (int s4 = 0; s4 < p.NCOL / 16; ++s4)
      for (int q = 0; q < 4; ++q) acc += lds[(4 * g) * p.S + 16 * w + j + (16 * s4 + q) * p.S];
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}
// gemm_dw B read: bb = buf + (16*nb0 + j)*S2 + 4g + t*16*S2 + 16*s4  (b128 read)
__global__ __launch_bounds__(512) void k_dwB(P p, float* out) {
  extern __shared__ float lds[];
  for (int i = threadIdx.x; i < 38000; i += blockDim.x) lds[i] = i;
  __syncthreads();
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15;
  v4f acc = {0, 0, 0, 0};
  for (int r = 0; r < REP; ++r)
    for (int t = 0; t < p.Wp / 16; ++t)
      for (int s4 = 0; s4 < p.NCOL / 16; ++s4)
        acc += *reinterpret_cast<const v4f*>(lds + j * p.S2 + 4 * g + t * 16 * p.S2 + 16 * s4);
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc[0] + acc[1] + acc[2] + acc[3];
}
// transposed-tile store: buf[(16*cb + 4g + i)*S + 16w + j]  (b32 write)
__global__ __launch_bounds__(512) void k_storefwd_t(P p, float* out) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  float v = lane;
  for (int r = 0; r < REP; ++r)
    for (int cb = 0; cb < p.NCOL / 16; ++cb)
      for (int i = 0; i < 4; ++i) {
        lds[(16 * cb + 4 * g + i) * p.S + 16 * w + j] = v;
        v += 1.f;
      }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = lds[threadIdx.x];
}
// transposed-tile recompute store: (16w + j)*S2 + 16*cb + 4g  (b128 write)
__global__ __launch_bounds__(512) void k_actbwd_t(P p, float* out) {
  extern __shared__ float lds[];
  const int lane = threadIdx.x & 63, g = lane >> 4, j = lane & 15, w = threadIdx.x >> 6;
  v4f v = {1.f * lane, 2, 3, 4};
  for (int r = 0; r < REP; ++r)
    for (int cb = 0; cb < p.NCOL / 16; ++cb) {
      *reinterpret_cast<v4f*>(lds + (16 * w + j) * p.S2 + 16 * cb + 4 * g) = v;
      v[1] += 1.f;
    }
  __syncthreads();
  out[blockIdx.x * blockDim.x + threadIdx.x] = lds[threadIdx.x];
}
// linear b128 read (reference: conflict-free)
__global__ __launch_bounds__(512) void k_lin(P p, float* out) {
  extern __shared__ float lds[];
  for (int i = threadIdx.x; i < 38000; i += blockDim.x) lds[i] = i;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  v4f acc = {0, 0, 0, 0};
  for (int r = 0; r < REP; ++r)
    for (int k = 0; k < 64; ++k) acc += *reinterpret_cast<const v4f*>(lds + 4 * lane + 256 * (k & 31));
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc[0] + acc[1] + acc[2] + acc[3];
}
// linear b32 read
__global__ __launch_bounds__(512) void k_lin32(P p, float* out) {
  extern __shared__ float lds[];
  for (int i = threadIdx.x; i < 38000; i += blockDim.x) lds[i] = i;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  float acc = 0;
  for (int r = 0; r < REP; ++r)
    for (int k = 0; k < 64; ++k) acc += lds[lane + 64 * (k & 31)];
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

int main() {
  P cfgs[2] = {{132, 132, 128, 128, 8}, {132, 100, 96, 112, 7}};
  float* out;
  if (hipMalloc(&out, 256 * 512 * 4) != hipSuccess) return 1;
  const size_t lds = 38000 * 4;
  (void)hipFuncSetAttribute((const void*)k_fwdB, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_storefwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_actbwd, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_dwA, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_dwB, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_lin, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_lin32, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_storefwd_t, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  (void)hipFuncSetAttribute((const void*)k_actbwd_t, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
  for (int c = 0; c < 2; ++c) {
    P p = cfgs[c];
    const int nthr = (p.Wp / 16) * 64;
    hipLaunchKernelGGL(k_fwdB, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_storefwd, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_actbwd, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_dwA, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_dwB, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_lin, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_lin32, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_storefwd_t, dim3(256), dim3(nthr), lds, 0, p, out);
    hipLaunchKernelGGL(k_actbwd_t, dim3(256), dim3(nthr), lds, 0, p, out);
    if (hipDeviceSynchronize() != hipSuccess) return 1;
  }
  hipError_t e = hipGetLastError();
  printf("ldsprobe done: %s\n", hipGetErrorString(e));
  return e != hipSuccess;
}
