// LDS bank microbenchmark for gfx950 (not part of the library): times
// 16-byte reads (ds_read_b128) and 8-byte atomic adds (ds_add_f64) for
// lane-to-address patterns, to fix the bank rules the schedule builder
// assumes.  Every address stays inside the 64 KiB array.
//
//   hipcc -O3 --offload-arch=gfx950 -Xclang -target-feature -Xclang -packed-fp32-ops \
//       paper_2202_04140_amd/csrc/lds_bank_probe.hip -o /tmp/lds_bank_probe && /tmp/lds_bank_probe
//
// Output: cycles per wave instruction per CU at 2.4 GHz (16 resident waves
// per CU, 4096 instructions each).
#include <hip/hip_runtime.h>
#include <cstdio>
constexpr int ND = 8192;      // doubles (64 KiB)
constexpr int ITERS = 4096;

// family 0 (slots): g groups per quarter, slot = (l%16)%g + 16*((l%16)/g) + 256*(l/16)  (max 1023)
// family 1 (doubles): stride k, d = k*lane (k <= 64: max 4032)
// family 2 (doubles): d = (lane % G) + 64*(lane / G)   (max 63 + 64*63 = 4095)
__device__ int pat(int fam, int prm, int lane) {
  if (fam == 0) {
    const int q = lane & 15;
    return 2 * ((q % prm) + 16 * (q / prm) + 256 * (lane >> 4));   // double index of the slot
  }
  if (fam == 1) return prm * lane;
  return (lane % prm) + 64 * (lane / prm);
}

template <int KIND>   // 0: b128 read of the slot at d (d even), 1: ds_add_f64 at d, 2: ds_add_f64 at d and d+1
__global__ void probe(int fam, int prm, double* out) {
  __shared__ double lds[ND];
  for (int i = threadIdx.x; i < ND; i += blockDim.x) lds[i] = i * 1e-3;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int d0 = pat(fam, prm, lane) + 512 * w;   // <= 4095 + 1536
  double acc = 0.0;
  for (int it = 0; it < ITERS; ++it) {
    int d = d0 + 256 * (it & 7);                 // <= 5631 + 1792 + 1 < ND
    asm volatile("" : "+v"(d));
    if (KIND == 0) {
      const double2 v = *reinterpret_cast<const double2*>(&lds[d & ~1]);
      acc += v.x + v.y;
    } else {
      atomicAdd(&lds[d], 1.0);
      if (KIND == 2) atomicAdd(&lds[d + 1], 1.0);
    }
  }
  __syncthreads();
  if (KIND) acc = lds[d0];
  out[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

int main() {
  const int blocks = 1024, threads = 256;
  double* out;
  (void)hipMalloc(&out, sizeof(double) * blocks * threads);
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  struct Case { int kind, fam, prm; };
  const Case cases[] = {
      {0, 0, 16}, {0, 0, 8}, {0, 0, 6}, {0, 0, 5}, {0, 0, 4}, {0, 0, 3}, {0, 0, 2}, {0, 0, 1},
      {2, 0, 16}, {2, 0, 8}, {2, 0, 6}, {2, 0, 5}, {2, 0, 4}, {2, 0, 3}, {2, 0, 2}, {2, 0, 1},
      {1, 1, 1}, {1, 1, 2}, {1, 1, 4}, {1, 1, 8}, {1, 1, 16}, {1, 1, 32}, {1, 1, 64},
      {1, 2, 4}, {1, 2, 8}, {1, 2, 16}, {1, 2, 32}, {1, 2, 64},
  };
  for (const Case& c : cases) {
    float best = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      (void)hipEventRecord(a);
      if (c.kind == 0) probe<0><<<blocks, threads>>>(c.fam, c.prm, out);
      if (c.kind == 1) probe<1><<<blocks, threads>>>(c.fam, c.prm, out);
      if (c.kind == 2) probe<2><<<blocks, threads>>>(c.fam, c.prm, out);
      (void)hipEventRecord(b);
      (void)hipEventSynchronize(b);
      float ms;
      (void)hipEventElapsedTime(&ms, a, b);
      if (ms < best) best = ms;
    }
    const double waves_per_cu = (double)blocks * threads / 64 / 256;
    const double instr = c.kind == 2 ? 2.0 : 1.0;
    printf("kind %d (%s) fam %d prm %2d: %.3f ms  %.2f cycles per wave instruction\n", c.kind,
           c.kind == 0 ? "read b128" : c.kind == 1 ? "add f64" : "add f64 x2 (re, im)", c.fam, c.prm, best,
           best * 2.4e6 / (waves_per_cu * ITERS * instr));
    fflush(stdout);
  }
  printf("status %s\n", hipGetErrorString(hipGetLastError()));
  return 0;
}
