// Launcher of the CPU emulation (hip_cpu.h).
#include "hip_cpu.h"

thread_local dim3 threadIdx;
thread_local dim3 blockIdx;
dim3 blockDim, gridDim;
thread_local int emu_tid;
EmuBlock *emu_blk;

void emu_launch(unsigned grid, unsigned block, std::function<void()> fn) {
    gridDim.x = grid;
    blockDim.x = block;
    for (unsigned b = 0; b < grid; ++b) {
        EmuBlock blk;
        std::barrier<> bar((std::ptrdiff_t)block);
        blk.bar = &bar;
        for (unsigned w = 0; w < (block + TC_WAVE - 1) / TC_WAVE; ++w) blk.waves.push_back(new EmuWave());
        emu_blk = &blk;
        std::vector<std::thread> th;
        for (unsigned t = 0; t < block; ++t)
            th.emplace_back([&, t, b]() {
                emu_tid = (int)t;
                threadIdx.x = t;
                blockIdx.x = b;
                fn();
            });
        for (auto &x : th) x.join();
        for (auto *w : blk.waves) delete w;
    }
}
