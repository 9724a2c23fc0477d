// ks_launch.h -- host-side launchers of the libksmul kernels (one per translation unit).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "ks_jobs.h"

namespace ks {

// Launch timing: a timed region of the host code hands the kernel launches of its thread a pair
// of events, which the first launch records at its start and the last at its end
// (hipExtLaunchKernelGGL: the dispatch's own timestamps, not those of the stream around it).
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
    bool used = false;
};
LaunchEvents &launch_events();  // this thread's pair (none outside timed regions)

template <typename K, typename... Args>
inline void ks_launch(K kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t s, Args... args) {
    LaunchEvents &ev = launch_events();
    if (ev.stop) {
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, ev.used ? nullptr : ev.start, ev.stop, 0u, args...);
        ev.used = true;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
    }
}

// ipt: limbs per thread of the carry-scan kernels, as planned (pack: SCAN_IPT_SINGLE or
// PACK_IPT_BATCH; recombination: SCAN_IPT_SINGLE or SCAN_IPT_BATCH);
// pack_w: the widest input coefficient (limbs) among the pack jobs
hipError_t launch_pack(const Launch<PackJob> &L, int ipt, int pack_w, hipStream_t s);
hipError_t launch_pack_anchor(const Launch<PackJob> &Lp, const Launch<AnchorJob> &La, int w_in, int ipt,
                              int pack_w, hipStream_t s);
hipError_t launch_normalize(const Launch<NormJob> &L, int ipt, bool dual, hipStream_t s);  // dual: paired jobs present
hipError_t launch_pack_small(const Launch<PackJob> &L, int ipt, int pack_w, hipStream_t s);
hipError_t launch_normalize_small(const Launch<NormJob> &L, int ipt, hipStream_t s);
hipError_t launch_mul_valu(const Launch<MulJob> &L, hipStream_t s);
hipError_t launch_mul_valu_wave(const Launch<MulJob> &L, hipStream_t s);
hipError_t launch_extract(const Launch<ExtractJob> &L, hipStream_t s);
hipError_t launch_anchor(const Launch<AnchorJob> &L, int w_in, hipStream_t s);
// lanes: the jobs' units are segments (batches), else blocks of CHAIN_TPB segments; nw = 0 only
// with lanes (jobs of several widths)
hipError_t launch_chain(const Launch<ChainJob> &L, int nw, bool lanes, hipStream_t s);
hipError_t launch_finish(const Launch<ChainJob> &L, int nw, hipStream_t s);
hipError_t launch_fill_zero(uint64_t *p, int64_t n, hipStream_t s);
hipError_t launch_digitize(const Launch<DigitJob> &L, hipStream_t s);
hipError_t launch_mul_mfma(const Launch<MfmaJob> &L, int rt, hipStream_t s);  // rt: tiles per block (4 or 8)
// one of the transform steps of integer products on the transform engine: 0 forward columns,
// 1 rows (both operands forward, the pointwise product, inverse), 2 inverse columns
// max_k1, max_k2: the longest columns and rows (log2 N1, log2 N2) among the launch's jobs
// (they size the steps' twiddle tables in LDS)
hipError_t launch_ntt_stage(int stage, const Launch<NttJob> &L, int max_k1, int max_k2, hipStream_t s);
hipError_t launch_ntt_join(const Launch<NttJoinJob> &L, hipStream_t s);
hipError_t launch_p2_eval(const P2Eval &E, hipStream_t s);
hipError_t launch_p2_readoff(const P2Readoff &R, hipStream_t s);
hipError_t launch_p2_glue(const P2Glue &G, hipStream_t s);  // two launches (chunk sums, then outputs)
hipError_t launch_p2_ext_eval(const P2ExtEval &E, hipStream_t s);
hipError_t launch_p2_ext_readoff(const P2ExtReadoff &R, hipStream_t s);
// polynomial-level Karatsuba of a batch: `tab` holds `count` KaraProd on the device
hipError_t launch_kara_split(const KaraProd *tab, int64_t count, int64_t max_h, const uint32_t *in, uint64_t *sub,
                             hipStream_t s);
hipError_t launch_kara_combine(const KaraProd *tab, int64_t count, int64_t max_out, const uint64_t *sub,
                               uint32_t *out, hipStream_t s);

}  // namespace ks
