// Batched AMP-PCG: many independent systems advanced in lockstep by the
// same three kernels per iteration.  Each work-group reads its (system,
// logical index) pair from a task table and runs the single-system stage
// code on that system's data with that system's work-group count G, so a
// system's reductions, controller decisions and state chain are exactly
// those of a single-system solve with G work-groups.  Systems that have
// stopped are dropped from the task table between batches of iterations;
// a stopped system still in the table passes its state through unchanged.
#pragma once

#include "amp_kernels.hpp"

namespace amp {

// One system of a batch (device-resident table, read-only during a solve).
struct SysDesc {
    Cfg c;              // g_stream = g_slice = g_pre = the system's G
    Sell A;
    Bufs B;
    St *st;             // the system's state slots
    double *bw;         // writable alias of B.b
    const double *b_in; // caller's right-hand side (n entries)
    double *x_io;       // caller's x0 in, solution out (n entries)
    int64_t n;
    int solo;           // solved by one work-group of k_batch_solo, not by the lockstep kernels
};

// A work-group's assignment; sys < 0 marks padding.  Besides (system,
// logical index) it carries what an iteration kernel's first loads need --
// the system's work-group count, state slots, partial arrays and residual
// window -- so that those loads wait only for the task, not for the
// system's descriptor.
struct Task {
    int sys, lb, g, pad;
    St *st;
    const double *part_res, *part_pre, *part_spmv, *ring;
};

// Every field of the task is used before the padding test, so the compiler
// loads the whole task at once instead of after the branch.
#define AMP_BATCH_TASK(sd, tasks, d, wg)                                                     \
    const Task t_ = (tasks)[xcd_block()];                                                    \
    pin((uint32_t)t_.lb ^ (uint32_t)t_.g ^ (uint32_t)(uintptr_t)t_.st ^                     \
        (uint32_t)(uintptr_t)t_.part_res ^ (uint32_t)(uintptr_t)t_.part_pre ^              \
        (uint32_t)(uintptr_t)t_.part_spmv ^ (uint32_t)(uintptr_t)t_.ring);                 \
    if (t_.sys < 0) return;                                                                  \
    const SysDesc &d = (sd)[t_.sys];                                                         \
    const Wg wg{t_.lb, t_.g}

// Copy b and x0 into the padded work vectors; lb 0 writes the initial state.
__global__ void __launch_bounds__(NT) k_batch_prep(const SysDesc *sd, const Task *tasks, St s0, int slot) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    int64_t lo, hi;
    block_range(d.n, NT, wg.lb, wg.G, lo, hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += NT) {
        d.bw[i] = d.b_in[i];
        d.B.x[i] = d.x_io[i];
    }
    if (wg.lb == 0 && threadIdx.x == 0) d.st[slot] = s0;
}

__global__ void __launch_bounds__(NTS) k_batch_init(const SysDesc *sd, const Task *tasks) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    init_stage<NTS>(d.A, d.B, wg);
}

__global__ void __launch_bounds__(NT) k_batch_precond(const SysDesc *sd, const Task *tasks, int si, int so) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    precond_stage(d.c, d.A, d.B, d.A.np, t_.st + si, t_.st + so, wg, Early{t_.part_res, t_.g, t_.ring, 0u});
}

// (the same block size and u_z specialisation as k_spmv, so a system's
// partial sums are those of its single solve; one chunk of slots per pass
// -- the order of the sums does not depend on it -- keeps the kernel within
// the register budget of 4 waves per SIMD)
template <int UZF>
__global__ void __launch_bounds__(NTP, 4) k_batch_spmv(const SysDesc *sd, const Task *tasks, int si, int so) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    spmv_stage<NTP, false, UZF, kChunk>(d.c, d.A, d.B, t_.st + si, t_.st + so, wg,
                                        Early{t_.part_pre, t_.g, nullptr, 0u});
}

__global__ void __launch_bounds__(NT) k_batch_update(const SysDesc *sd, const Task *tasks, int si, int so) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    update_stage(d.c, d.B, d.A.np, t_.st + si, t_.st + so, wg, Early{t_.part_spmv, t_.g, nullptr, 0u});
}

__global__ void __launch_bounds__(NTS) k_batch_true_res(const SysDesc *sd, const Task *tasks, int mode, int si,
                                                       int so) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    true_res_stage<NTS>(d.c, d.A, d.B, mode, d.st + si, d.st + so, wg);
}

// Partials of ||b - A x||^2 in FP64 (no state involved).
__global__ void __launch_bounds__(NTS) k_batch_report(const SysDesc *sd, const Task *tasks) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    double st = 0.0, ss = 0.0, mr = 0.0;
    true_res_body<64, NTS>(d.A, d.B, wg, false, st, ss, mr);
    st = block_sum<NTS>(st);
    if (threadIdx.x == 0) d.B.part_res[wg.lb] = st;
}

// One work-group per system: the fixed-order total of its report partials.
__global__ void __launch_bounds__(NT) k_batch_reduce_report(const SysDesc *sd, int nsys, double *out) {
    const int sys = blockIdx.x;
    if (sys >= nsys) return;
    const double t = reduce_sum(sd[sys].B.part_res, sd[sys].c.g_stream);
    if (threadIdx.x == 0) out[sys] = t;
}

// State slot `slot` of every lockstep system (of every single-work-group
// system when slot is ST_FIN) into one array, for one host copy.
__global__ void __launch_bounds__(NT) k_batch_gather(const SysDesc *sd, int nsys, int slot, St *out) {
    const int sys = blockIdx.x * NT + threadIdx.x;
    if (sys < nsys && (sd[sys].solo != 0) == (slot == ST_FIN)) out[sys] = sd[sys].st[slot];
}

// The small systems: one work-group each runs its whole solve.
__global__ void __launch_bounds__(NT) k_batch_solo(const SysDesc *sd, const int *list, int cap) {
    const SysDesc &d = sd[list[blockIdx.x]];
    solo_solve<false>(d.c, d.A, d.B, d.st, cap);
}

__global__ void __launch_bounds__(NT) k_batch_copy_out(const SysDesc *sd, const Task *tasks) {
    AMP_BATCH_TASK(sd, tasks, d, wg);
    int64_t lo, hi;
    block_range(d.n, NT, wg.lb, wg.G, lo, hi);
    for (int64_t i = lo + threadIdx.x; i < hi; i += NT) d.x_io[i] = d.B.x[i];
}

}  // namespace amp
