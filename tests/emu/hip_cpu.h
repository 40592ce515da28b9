// CPU emulation of the few HIP device features the fold kernels of
// tc_count_mid.hip use, for a host test of their logic.  Every lane of a
// workgroup is one OS thread; workgroups run one after another.  The GPU
// runs a wavefront's lanes in lockstep; here lanes only meet at the
// wavefront barrier, which the kernels place at every phase boundary whose
// LDS accesses cross lanes (wave_lds_sync).  Shuffles exchange through
// per-wavefront slots between two barriers, so every lane of a wavefront
// must reach each shuffle the same number of times.
#pragma once
#include <algorithm>
#include <atomic>
#include <barrier>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <functional>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __shared__ static
#define __forceinline__ inline
#define __launch_bounds__(...)
#define TC_WAVE 64

using std::min;

struct dim3 { unsigned x = 1, y = 1, z = 1; };
struct uint2 { uint32_t x, y; };
struct uint4 { uint32_t x, y, z, w; };
inline uint2 make_uint2(uint32_t a, uint32_t b) { return uint2{a, b}; }
inline uint4 make_uint4(uint32_t a, uint32_t b, uint32_t c, uint32_t d) { return uint4{a, b, c, d}; }

extern thread_local dim3 threadIdx;
extern thread_local dim3 blockIdx;
extern dim3 blockDim, gridDim;
extern thread_local int emu_tid;

struct EmuWave {
    std::barrier<> bar{TC_WAVE};
    uint64_t slots[TC_WAVE];
};
struct EmuBlock {
    std::vector<EmuWave *> waves;
    std::barrier<> *bar = nullptr;  // the workgroup barrier
};
extern EmuBlock *emu_blk;

inline int __lane_id() { return emu_tid % TC_WAVE; }
inline void __syncthreads() { emu_blk->bar->arrive_and_wait(); }
inline void __builtin_amdgcn_wave_barrier() { emu_blk->waves[emu_tid / TC_WAVE]->bar.arrive_and_wait(); }
#define __builtin_amdgcn_fence(order, scope) std::atomic_thread_fence(std::memory_order_seq_cst)

// lane l receives the value of lane src(l) (all lanes of the wavefront take part)
inline uint64_t emu_exchange(uint64_t v, int src) {
    EmuWave &w = *emu_blk->waves[emu_tid / TC_WAVE];
    w.slots[emu_tid % TC_WAVE] = v;
    w.bar.arrive_and_wait();
    const uint64_t r = w.slots[src];
    w.bar.arrive_and_wait();
    return r;
}
template <typename T> inline T __shfl_xor(T x, int m, int width = TC_WAVE) {
    uint64_t u = 0;
    std::memcpy(&u, &x, sizeof(T));
    const int l = __lane_id();
    const uint64_t r = emu_exchange(u, (l & ~(width - 1)) | ((l ^ m) & (width - 1)));
    T o;
    std::memcpy(&o, &r, sizeof(T));
    return o;
}

template <typename T> inline T __shfl_up(T x, unsigned d, int width = TC_WAVE) {
    uint64_t u = 0;
    std::memcpy(&u, &x, sizeof(T));
    const int l = __lane_id(), base = l & ~(width - 1);
    const uint64_t r = emu_exchange(u, l - base >= (int)d ? l - (int)d : l);
    T o;
    std::memcpy(&o, &r, sizeof(T));
    return o;
}

inline int __popc(uint32_t x) { return __builtin_popcount(x); }
// v_bfe_u32: offset and width from the low 5 bits of their operands; width 0 gives 0
inline uint32_t __builtin_amdgcn_ubfe(uint32_t x, uint32_t off, uint32_t width) {
    const uint32_t o = off & 31u, w = width & 31u;
    return w == 0 ? 0u : (x >> o) & ((1u << w) - 1u);
}
inline uint32_t atomicOr(uint32_t *p, uint32_t v) { return std::atomic_ref<uint32_t>(*p).fetch_or(v); }
inline uint32_t __umul24(uint32_t a, uint32_t b) { return (a & 0xFFFFFFu) * (b & 0xFFFFFFu); }
inline uint32_t __builtin_amdgcn_alignbit(uint32_t hi, uint32_t lo, uint32_t s) {
    return (uint32_t)(((((uint64_t)hi) << 32) | lo) >> (s & 31u));
}
inline uint32_t atomicAdd(uint32_t *p, uint32_t v) { return std::atomic_ref<uint32_t>(*p).fetch_add(v); }

// Runs fn on grid workgroups of block threads, one workgroup at a time.
void emu_launch(unsigned grid, unsigned block, std::function<void()> fn);
