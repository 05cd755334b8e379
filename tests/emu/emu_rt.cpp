// The fake HIP runtime of the emulation: host memory as device memory,
// buffer loads with the hardware's range rule, pseudo-random event times.
#include <hip/hip_runtime.h>
#include <cstdlib>
#include <random>
dim3 blockIdx, threadIdx, blockDim, gridDim;
static std::mt19937 rng(std::getenv("EMU_SEED") ? atoi(std::getenv("EMU_SEED")) : 1);
static long n_loads = 0;

static const char *load_at(emu_rsrc r, int voff, int soff, unsigned size, bool &zero) {
  const uint64_t off = (uint64_t)(uint32_t)voff + (uint64_t)(uint32_t)soff;
  if (off >> 32) {
    fprintf(stderr, "EMU: buffer offset wraps 32 bits: voff %u soff %u base %p nrec %u\n",
            (unsigned)voff, (unsigned)soff, (const void *)r.base, r.nrec);
    abort();
  }
  zero = r.nrec != 0xFFFFFFFFu && off + size > r.nrec;
  ++n_loads;
  return r.base + off;
}
uint64_t emu_buffer_load64(emu_rsrc r, int voff, int soff) {
  bool zero; const char *p = load_at(r, voff, soff, 8, zero);
  if (zero) return 0;
  uint64_t v; memcpy(&v, p, 8); return v;
}
uint32_t emu_buffer_load32(emu_rsrc r, int voff, int soff) {
  bool zero; const char *p = load_at(r, voff, soff, 4, zero);
  if (zero) return 0;
  uint32_t v; memcpy(&v, p, 4); return v;
}
hipError_t hipMalloc(void **p, size_t n) {
  size_t m = (n + 255) / 256 * 256; if (!m) m = 256;
  *p = aligned_alloc(256, m);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void *p) { free(p); return hipSuccess; }
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) { memmove(d, s, n); return hipSuccess; }
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind k, hipStream_t) { return hipMemcpy(d, s, n, k); }
hipError_t hipMemset(void *d, int v, size_t n) { memset(d, v, n); return hipSuccess; }
hipError_t hipMemsetAsync(void *d, int v, size_t n, hipStream_t) { memset(d, v, n); return hipSuccess; }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipDeviceSynchronize() { return hipSuccess; }
struct emu_event { int x; };
hipError_t hipEventCreate(hipEvent_t *e) { *e = new emu_event{0}; return hipSuccess; }
hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
  *ms = 1.0f + std::uniform_real_distribution<float>(0.f, 1.f)(rng); return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t e) { delete e; return hipSuccess; }
struct emu_graph { int x; };
struct emu_graph_exec { int x; };
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipSuccess; }
hipError_t hipGraphDestroy(hipGraph_t g) { delete g; return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t g) { delete g; return hipSuccess; }
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode) { return hipSuccess; }
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *g) { *g = new emu_graph{0}; return hipSuccess; }
hipError_t hipGraphInstantiate(hipGraphExec_t *e, hipGraph_t, void *, void *, size_t) { *e = new emu_graph_exec{0}; return hipSuccess; }
struct emu_stream { int x; };
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) { *s = new emu_stream{0}; return hipSuccess; }
hipError_t hipStreamDestroy(hipStream_t s) { delete s; return hipSuccess; }
hipError_t hipGetDevice(int *d) { *d = 0; return hipSuccess; }
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t, int) { *v = 65536; return hipSuccess; }
hipError_t hipGetLastError() { return hipSuccess; }
const char *hipGetErrorString(hipError_t) { return "emu error"; }
static double emu_symbol[1 << 20];
hipError_t hipGetSymbolAddress(void **p, const void *) { *p = emu_symbol; return hipSuccess; }
extern "C" long emu_loads() { return n_loads; }
