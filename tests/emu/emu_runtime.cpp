// Test infrastructure: the scheduler behind tests/emu/hip/hip_runtime.h (see there).  Threads
// of a block are coroutines on stacks of their own, switched by a few instructions that save
// and restore the callee-saved registers (x86-64 System V); AddressSanitizer is told about
// every stack switch.
#include <hip/hip_runtime.h>

#include <sys/mman.h>

#include <cstdio>
#include <cstdlib>
#include <memory>
#include <vector>

#if defined(__has_feature)
#if __has_feature(address_sanitizer)
#define EMU_ASAN 1
#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#endif
#endif

// Saves the callee-saved registers on the current stack, stores the stack pointer in *save,
// switches to the stack `next` and restores that stack's registers.
extern "C" void emu_switch(void** save, void* next);
asm(R"(
    .text
    .globl emu_switch
    .type emu_switch, @function
emu_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_switch, .-emu_switch
)");

namespace emu {

namespace {

constexpr int kWave = 64;
constexpr int kMaxThreads = 1024;
constexpr size_t kStack = 512 * 1024;
constexpr size_t kMaxLds = 160 * 1024;

enum State : int { kRunnable = 0, kWaveWait, kBarrierWait, kDone };

}  // namespace

struct Lane {
    void* sp = nullptr;
    char* stack = nullptr;
    dim3 tid;
    int state = kDone;
    int op = 0, param = 0, width = 64;
    const void* site = nullptr;
    uint64_t in = 0, out = 0;
    bool deposited = false;
    void* fake = nullptr;
};

namespace {

Lane g_lanes[kMaxThreads];
int g_nlanes = 0;
Lane* g_cur = nullptr;
void* g_sched_sp = nullptr;
void* g_sched_fake = nullptr;
const void* g_main_bottom = nullptr;
size_t g_main_size = 0;
dim3 g_block, g_grid, g_bdim;
std::unique_ptr<unsigned char[]> g_dyn;
const std::function<void()>* g_body = nullptr;
hipError_t g_err = hipSuccess;
uint64_t g_inactive_reads = 0, g_launches = 0, g_blocks = 0;

[[noreturn]] void fail(const char* what, const void* site = nullptr)
{
    std::fprintf(stderr, "[emu] %s (block %u, thread %u, site %p)\n", what, g_block.x,
                 g_cur ? g_cur->tid.x : 0u, site);
    std::fflush(stderr);
    std::abort();
}

void to_scheduler(Lane* l)
{
#ifdef EMU_ASAN
    __sanitizer_start_switch_fiber(l->state == kDone ? nullptr : &l->fake, g_main_bottom,
                                   g_main_size);
#endif
    emu_switch(&l->sp, g_sched_sp);
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(l->fake, &g_main_bottom, &g_main_size);
#endif
}

void lane_main()
{
    Lane* l = g_cur;
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &g_main_bottom, &g_main_size);
#endif
    (*g_body)();
    l->state = kDone;
    to_scheduler(l);
    fail("a finished thread was resumed");
}

void resume(Lane* l)
{
    g_cur = l;
#ifdef EMU_ASAN
    __sanitizer_start_switch_fiber(&g_sched_fake, l->stack, kStack);
#endif
    emu_switch(&g_sched_sp, l->sp);
#ifdef EMU_ASAN
    __sanitizer_finish_switch_fiber(g_sched_fake, nullptr, nullptr);
#endif
    g_cur = nullptr;
}

// Completes the wave operation the lanes in `act` (one wave, same call site) wait at.
void resolve(Lane* w, const std::vector<int>& act)
{
    const Lane& a0 = w[act[0]];
    uint64_t active = 0;
    for (int i : act) active |= 1ull << i;
    if (a0.op == kOpBallot) {
        uint64_t m = 0;
        for (int i : act)
            if (w[i].in & 1u) m |= 1ull << i;
        for (int i : act) w[i].out = m;
    } else if (a0.op == kOpWaveBarrier) {
        for (int i : act) w[i].out = 0;
    } else {
        for (int i : act) {
            const int width = w[i].width, seg = i & ~(width - 1), p = w[i].param;
            int src = i;
            switch (w[i].op) {
                case kOpShfl: src = seg + (p & (width - 1)); break;
                case kOpShflUp: src = (i - seg) >= p ? i - p : i; break;
                case kOpShflDown: src = (i - seg) + p < width ? i + p : i; break;
                case kOpShflXor: src = i ^ p; break;
                default: fail("unknown wave operation", w[i].site);
            }
            if (src < 0 || src >= kWave) src = i;
            if (!((active >> src) & 1ull)) ++g_inactive_reads;  // stale register on the device
            w[i].out = w[src].in;
        }
    }
    for (int i : act) {
        w[i].deposited = false;
        w[i].state = kRunnable;
    }
}

void run_block()
{
    const int n = g_nlanes;
    for (int t = 0; t < n; ++t) {
        Lane& l = g_lanes[t];
        if (!l.stack) {
            void* s = mmap(nullptr, kStack, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS,
                           -1, 0);
            if (s == MAP_FAILED) fail("no memory for a thread stack");
            l.stack = static_cast<char*>(s);
        }
        l.tid = dim3(t % g_bdim.x, (t / g_bdim.x) % g_bdim.y, t / (g_bdim.x * g_bdim.y));
        l.state = kRunnable;
        l.in = l.out = 0;
        l.deposited = false;
        l.fake = nullptr;
        // a fresh stack as emu_switch leaves one: six saved registers, then lane_main as the
        // return address, entered with the stack aligned as after a call
        uintptr_t top = (reinterpret_cast<uintptr_t>(l.stack) + kStack) & ~uintptr_t(15);
        void** sp = reinterpret_cast<void**>(top - 64);
        for (int r = 0; r < 6; ++r) sp[r] = nullptr;
        sp[6] = reinterpret_cast<void*>(&lane_main);
        sp[7] = nullptr;
        l.sp = sp;
    }
    for (;;) {
        for (int t = 0; t < n; ++t)
            if (g_lanes[t].state == kRunnable) resume(&g_lanes[t]);
        bool all_done = true, progressed = false;
        for (int w0 = 0; w0 < n; w0 += kWave) {
            Lane* w = g_lanes + w0;
            const int nw = std::min(kWave, n - w0);
            std::vector<int> act;
            for (int i = 0; i < nw; ++i) {
                if (w[i].state != kDone) all_done = false;
                if (w[i].state == kWaveWait) act.push_back(i);
            }
            if (act.empty()) continue;
            for (int i : act)
                if (w[i].site != w[act[0]].site || w[i].op != w[act[0]].op)
                    fail("lanes of one wave wait at different wave operations", w[i].site);
            resolve(w, act);
            progressed = true;
        }
        if (all_done) break;
        if (progressed) continue;
        // no wave operation pending: every live thread waits at the block barrier
        for (int t = 0; t < n; ++t) {
            if (g_lanes[t].state == kBarrierWait) {
                g_lanes[t].state = kRunnable;
            } else if (g_lanes[t].state != kDone) {
                fail("threads neither at the barrier nor finished");
            }
        }
    }
}

}  // namespace

Lane* cur() { return g_cur; }
const dim3& thread_idx() { return g_cur->tid; }
const dim3& block_idx() { return g_block; }
const dim3& block_dim() { return g_bdim; }
const dim3& grid_dim() { return g_grid; }
void* dyn_lds() { return g_dyn.get(); }
hipError_t& last_error() { return g_err; }

void lds_fresh(void* p, size_t bytes)
{
    static std::vector<std::pair<void*, uint64_t>> seen;  // array, serial of the block that filled it
    for (auto& s : seen) {
        if (s.first == p) {
            if (s.second == g_blocks) return;
            s.second = g_blocks;
            std::memset(p, 0xA5, bytes);
            return;
        }
    }
    seen.emplace_back(p, g_blocks);
    std::memset(p, 0xA5, bytes);
}

uint64_t wave_op(int op, uint64_t bits, int param, int width, const void* site)
{
    Lane* l = g_cur;
    if (!l) fail("wave operation outside a kernel");
    if (width <= 0 || width > kWave || (width & (width - 1))) fail("bad shuffle width", site);
    l->op = op;
    l->param = param;
    l->width = width;
    l->site = site;
    l->in = bits;
    l->deposited = true;
    l->state = kWaveWait;
    to_scheduler(l);
    return l->out;
}

void sync_block(const void* site)
{
    Lane* l = g_cur;
    if (!l) fail("__syncthreads outside a kernel");
    l->site = site;
    l->state = kBarrierWait;
    to_scheduler(l);
}

void launch(const dim3& grid, const dim3& block, size_t dyn_lds_bytes,
            const std::function<void()>& body)
{
    const uint64_t nt = (uint64_t)block.x * block.y * block.z;
    if (nt == 0 || nt > (uint64_t)kMaxThreads || dyn_lds_bytes > kMaxLds) {
        g_err = hipErrorInvalidValue;
        return;
    }
    if (g_cur) fail("kernel launched from a kernel");
    ++g_launches;
    g_grid = grid;
    g_bdim = block;
    g_nlanes = (int)nt;
    g_body = &body;
    // dynamic LDS holds no defined values when a block starts
    g_dyn.reset(new unsigned char[dyn_lds_bytes ? dyn_lds_bytes : 1]);
    for (uint32_t z = 0; z < grid.z; ++z)
        for (uint32_t y = 0; y < grid.y; ++y)
            for (uint32_t x = 0; x < grid.x; ++x) {
                g_block = dim3(x, y, z);
                std::memset(g_dyn.get(), 0xA5, dyn_lds_bytes);
                run_block();
                ++g_blocks;
            }
    g_body = nullptr;
}

}  // namespace emu

// Counters of the emulation: launches, blocks, shuffles that read an inactive lane.
extern "C" void emu_counters(uint64_t* out3)
{
    out3[0] = emu::g_launches;
    out3[1] = emu::g_blocks;
    out3[2] = emu::g_inactive_reads;
}
