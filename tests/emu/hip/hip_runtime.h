// Host emulation of the parts of the HIP runtime the library's host code and
// the emulated kernels use. Device memory is host memory (malloc), so
// AddressSanitizer checks every access the emulated kernels make.
#pragma once
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <cstdio>
#include <cstddef>
#include <cmath>
using std::sqrt; using std::fabs; using std::fmax; using std::fmin;

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(x)
#define __shared__ static
#define HIP_SYMBOL(x) (&(x))

typedef enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 } hipError_t;
typedef struct emu_stream *hipStream_t;
typedef struct emu_event *hipEvent_t;
typedef struct emu_graph *hipGraph_t;
typedef struct emu_graph_exec *hipGraphExec_t;
typedef enum { hipMemcpyHostToDevice, hipMemcpyDeviceToHost, hipMemcpyDeviceToDevice, hipMemcpyDefault } hipMemcpyKind;
typedef enum { hipDeviceAttributeMaxSharedMemoryPerBlock } hipDeviceAttribute_t;
typedef enum { hipStreamCaptureModeGlobal, hipStreamCaptureModeThreadLocal } hipStreamCaptureMode;
#define hipStreamNonBlocking 1

struct dim3 {
  unsigned x, y, z;
  dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
extern dim3 blockIdx, threadIdx, blockDim, gridDim;

struct emu_rsrc { const char *base; uint32_t nrec; };
typedef emu_rsrc __amdgpu_buffer_rsrc_t;
uint64_t emu_buffer_load64(emu_rsrc r, int voff, int soff);
uint32_t emu_buffer_load32(emu_rsrc r, int voff, int soff);
#define __builtin_amdgcn_readfirstlane(x) (x)
#define __builtin_amdgcn_make_buffer_rsrc(p, stride, nrec, flags) (emu_rsrc{(const char *)(p), (uint32_t)(nrec)})
#define __builtin_amdgcn_raw_buffer_load_b64(r, v, s, a) emu_buffer_load64((r), (v), (s))
#define __builtin_amdgcn_raw_buffer_load_b32(r, v, s, a) emu_buffer_load32((r), (v), (s))

hipError_t hipMalloc(void **p, size_t n);
hipError_t hipFree(void *p);
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t st = 0);
hipError_t hipMemset(void *d, int v, size_t n);
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t st = 0);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipDeviceSynchronize();
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = 0);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipGraphLaunch(hipGraphExec_t g, hipStream_t s);
hipError_t hipGraphDestroy(hipGraph_t g);
hipError_t hipGraphExecDestroy(hipGraphExec_t g);
hipError_t hipStreamBeginCapture(hipStream_t s, hipStreamCaptureMode m);
hipError_t hipStreamEndCapture(hipStream_t s, hipGraph_t *g);
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t g, void *, void *, size_t);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned f);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipGetDevice(int *d);
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int d);
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipGetSymbolAddress(void **p, const void *sym);

// one thread at a time: blockIdx and threadIdx set before each call
template <typename F>
inline void emu_launch(dim3 grid, unsigned block, F f) {
  gridDim = grid;
  blockDim = dim3(block);
  for (unsigned by = 0; by < grid.y; ++by)
    for (unsigned bx = 0; bx < grid.x; ++bx) {
      blockIdx = dim3(bx, by);
      for (unsigned tx = 0; tx < block; ++tx) {
        threadIdx = dim3(tx);
        f();
      }
    }
}
