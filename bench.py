#!/usr/bin/env python3
"""Benchmark of the hx hot path on one MI355X.

Workload: a 1D periodic heat stencil over 2^28 fp32 cells split into 64
partitions of 4 Mi cells, r = 0.25, 50 steps (Sec. V-A.2 / Algorithm 1 with
the Sec. V-A.1 stencil).

`value` is the throughput of the whole 50-step run with the partitions
resident in HBM (laid out back to back in one arena): each pass of 50 fused
steps is one node of the future graph, launched as one batched kernel over
all 64 partitions with every partition's halos read from its neighbours.  One
bench "step" is the whole 50-step run over the whole array.  The pass runs in
the batched plan's form, pass depth and walk that the library's autotuner
picks: the direct form (the tile kernel stepping in registers, vector ALUs
only) or the propagator form (the 50 steps as one convolution with the
50-step propagator on the matrix cores; see `config.update_form`).  The
default warm-up (100 passes, about 40 ms) runs before the timed region so
that the card's clocks have settled: in the first 50-100 back-to-back passes
after an idle spell its power management first lets them run fast, then pulls
them down, then settles (per-launch times are in the log).

The same configuration host to host (pinned host partitions, per-partition
H2D -> 50-step kernel -> D2H, overlapped) is `host_to_host`, with the copy
overlap it reaches and the host link's own rates (`host_link`: H2D alone, D2H
alone, both together).  The PCIe-inclusive throughput is never `value`.

Printed: one JSON line with the throughput, the roofline of the timed kernel
(per-launch durations from HIP events recorded on its stream in the timed
region), the error of one pass against the oracle on every cell, the oracle's
CPU throughput (the headline workload, and a bounded sample of every other
workload), and the side measurements the metric names: both forms of the
pass, the per-partition future graph, the plain one-launch-per-partition-
per-step form, the 2D host-to-host pipeline, the 4096-problem batched driver,
the fp64, 2D and adjoint workloads, the partition-benchmark overhead against
raw HIP streams, and a one-pass device copy (the copy ceiling, and the
calibration of the HBM counters).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK = 8.0e12            # bytes/s, MI355X HBM3E
VALU_F32_PEAK = 157.3e12     # flop/s: 256 CU x 128 FP32 lanes/clk x 2 (FMA) x 2.4 GHz
MFMA_16BIT_PEAK = 2.5e15     # flop/s, dense bf16 and fp16 matrix cores
FLOPS_PER_UPDATE_1D = 3      # rescaled update w' = fma(b, l + rt, w): one add + one fma
BYTES_PER_CELL_PASS = 8      # one fp32 read + one fp32 write per cell per pass
MFMA_FLOPS_PER_CHUNK = 6 * 32 * 32 * 16 * 2   # span walk: six bf16 32x32x16 products per chunk
MFMA_FLOPS_PER_CHUNK_IL = 3 * 32 * 32 * 16 * 2  # block/interleaved walks: three fp16 products
ROOT = os.path.dirname(os.path.abspath(__file__))
# per form: the committed counter summary of its kernel and the sources it is built from
KERNELS = {
    "direct": ("stencil1d_flat_2p28_fp32_traffic.md",
               ("paper_1810_11482_amd/csrc/hx_stencil1d.hip",
                "paper_1810_11482_amd/csrc/hx_internal.h")),
    "propagator": ("prop1d_2p28_fp32_traffic.md",
                   ("paper_1810_11482_amd/csrc/hx_prop1d.hip",
                    "paper_1810_11482_amd/csrc/hx_internal.h")),
    "propagator_il": ("prop1d_il_2p28_fp32_traffic.md",
                      ("paper_1810_11482_amd/csrc/hx_prop1d.hip",
                       "paper_1810_11482_amd/csrc/hx_internal.h")),
    "propagator_bw": ("prop1d_bw_2p28_fp32_traffic.md",
                      ("paper_1810_11482_amd/csrc/hx_prop1d.hip",
                       "paper_1810_11482_amd/csrc/hx_internal.h")),
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def intervals_union(iv):
    iv = sorted(iv)
    out = []
    for a, b in iv:
        if out and a <= out[-1][1]:
            out[-1][1] = max(out[-1][1], b)
        else:
            out.append([a, b])
    return out


def measure_len(iv):
    return sum(b - a for a, b in iv)


def intersect_len(u1, u2):
    i = j = 0
    tot = 0.0
    while i < len(u1) and j < len(u2):
        a = max(u1[i][0], u2[j][0])
        b = min(u1[i][1], u2[j][1])
        if a < b:
            tot += b - a
        if u1[i][1] < u2[j][1]:
            i += 1
        else:
            j += 1
    return tot


def kernel_source_hash(form):
    import hashlib
    h = hashlib.sha256()
    for f in KERNELS[form][1]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(form):
    """HBM bytes per launch of the form's kernel from the committed rocprofv3
    counter summary, or None when the kernel sources changed since it was taken."""
    try:
        text = open(os.path.join(ROOT, "profiles", KERNELS[form][0])).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.startswith("- "):
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_hash") != kernel_source_hash(form):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


class Partitioned:
    """Device state of the partitioned workload: pinned host input, and two
    ping-pong arenas (one allocation each) whose partitions are non-owning
    buffer views, so the 64 partitions are laid out back to back in HBM."""

    def __init__(self, hx, ctx, n, parts, steps, r):
        self.hx, self.ctx = hx, ctx
        self.n, self.parts, self.steps, self.r = n, parts, steps, r
        import workloads
        self.bounds = workloads.partition_bounds(n, parts)
        self.sizes = [s for _, s in self.bounds]
        self.host_in = hx.hx_host_alloc(ctx, n * 4)
        self.host_out = hx.hx_host_alloc(ctx, n * 4)
        arr = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * n).from_address(self.host_in))
        workloads.partitioned1d_u0(workloads.Partitioned1D(n=n, parts=parts, steps=steps, r=r),
                                   out=arr)
        self.u0 = arr
        self.arena_a = hx.hx_buffer_create(ctx, n * 4)
        self.arena_b = hx.hx_buffer_create(ctx, n * 4)
        pa, _ = hx.hx_buffer_ptr(ctx, self.arena_a)
        pb, _ = hx.hx_buffer_ptr(ctx, self.arena_b)
        self.A = [hx.hx_buffer_wrap(ctx, pa + o * 4, s * 4) for o, s in self.bounds]
        self.B = [hx.hx_buffer_wrap(ctx, pb + o * 4, s * 4) for o, s in self.bounds]
        self.reset()
        self.last = 0

    def reset(self):
        """Upload the initial state into arena A (partition by partition)."""
        hx, ctx = self.hx, self.ctx
        evs = []
        for (o, s), b in zip(self.bounds, self.A):
            d = hx.hx_copy_desc(hx.HX_H2D, self.host_in + o * 4, b, 0, 0, 0, s * 4)
            evs.append(hx.hx_copy_async(ctx, d))
        w = hx.hx_when_all(ctx, evs)
        assert hx.hx_wait(ctx, w) == hx.HX_OK
        for e in evs + [w]:
            hx.hx_event_release(ctx, e)
        self.cur_in_a = True

    def step(self, mode, time_block, cpl=0, nodes=False):
        hx = self.hx
        src, dst = (self.A, self.B) if self.cur_in_a else (self.B, self.A)
        d = hx.partitioned_desc(hx.HX_F32, self.sizes, src, dst, self.steps, self.r,
                                periodic=True, mode=mode, time_block=time_block,
                                cells_per_lane=cpl)
        ev, in_b, node_evs = hx.hx_run_partitioned(self.ctx, d, deps=[self.last] if self.last else [],
                                                   node_events=nodes)
        if self.last:
            hx.hx_event_release(self.ctx, self.last)
        self.last = ev
        if in_b:
            self.cur_in_a = not self.cur_in_a
        return node_evs

    def wait(self):
        st = self.hx.hx_wait(self.ctx, self.last)
        assert st == self.hx.HX_OK, self.hx.hx_last_error(self.ctx)

    def current(self):
        return self.A if self.cur_in_a else self.B


def time_steps(P, k, mode, tb, cpl, nodes=False):
    import torch
    P.wait() if P.last else None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    all_nodes = []
    for _ in range(k):
        ne = P.step(mode, tb, cpl, nodes=nodes)
        if ne:
            all_nodes.extend(ne)
    P.wait()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / k, all_nodes


class BatchedPass:
    """The partitioned run in its batched form: every pass of `tb` steps is one
    node of the future graph, launched as one batched kernel over all
    partitions (each partition's halos, `hw` >= tb cells, read from its
    neighbours' views), and chained on the previous pass.  form: the batched
    plan's direct form (tile geometry `cpl`) or its propagator form (`span`
    blocks per wave, 0 = the plan's choice)."""

    def __init__(self, hx, ctx, P, tb, cpl, form=0, span=0, hw=None, wpg=0, grid=-1):
        self.hx, self.ctx, self.P, self.tb, self.cpl = hx, ctx, P, tb, cpl
        hw = tb if hw is None else hw
        self.plans = []
        for src, dst in ((P.A, P.B), (P.B, P.A)):
            segs = []
            for p in range(P.parts):
                lp, rp = (p - 1) % P.parts, (p + 1) % P.parts
                segs.append(hx.segment(inp=src[p], out=dst[p], n=P.sizes[p], r=P.r,
                                       bc_lo=hx.HX_BC_GHOST, bc_hi=hx.HX_BC_GHOST,
                                       halo_lo=src[lp], halo_lo_offset=(P.sizes[lp] - hw) * 4,
                                       halo_hi=src[rp], halo_width=hw))
            self.plans.append(hx.hx_plan_create_batched(ctx, hx.HX_F32, tb, segs,
                                                        hx.HX_BATCH_PERSISTENT, cells_per_lane=cpl,
                                                        waves_per_group=wpg,
                                                        grid_waves_per_cu=grid, form=form,
                                                        span_blocks=span))
        self.passes = P.steps // tb
        assert self.passes * tb == P.steps, "the time block must divide the step count"

    def run(self, nsteps, keep=None):
        """Queue nsteps bench steps; launch events go to `keep` when given."""
        hx, P = self.hx, self.P
        for _ in range(nsteps * self.passes):
            plan = self.plans[0 if P.cur_in_a else 1]
            ev = hx.hx_launch_batched(self.ctx, plan, deps=[P.last] if P.last else [])
            if keep is not None:
                keep.append(ev)
            elif P.last:
                hx.hx_event_release(self.ctx, P.last)
            P.last = ev
            P.cur_in_a = not P.cur_in_a

    def close(self):
        for pl in self.plans:
            self.hx.hx_plan_destroy(self.ctx, pl)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    # the card's clocks settle over the first 50-100 back-to-back passes after
    # an idle spell (power management): the warm-up covers that transient
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--log2n", type=int, default=28)
    ap.add_argument("--parts", type=int, default=64)
    ap.add_argument("--cells-per-lane", type=int, default=0, help="0 = pick by a short sweep")
    ap.add_argument("--form", choices=("auto", "direct", "propagator"), default="auto",
                    help="form of the headline pass; auto = the faster in a short sweep")
    ap.add_argument("--span-blocks", type=int, default=0,
                    help="propagator form: 1024-cell blocks per wave, -1 = the interleaved "
                         "walk, -2 = the block walk, 0 = sweep the walks")
    ap.add_argument("--streams", type=int, default=4,
                    help="compute streams of the context (the per-partition graph spreads its "
                         "nodes over them)")
    ap.add_argument("--legs",
                    default="graph,plain,pipeline2d,batched,fp64,2d,adjoint,overhead,copy,"
                            "cpu",
                    help="comma list of side legs (the host-to-host run and the host-link "
                         "rates always run): graph (the per-partition future graph), "
                         "plain, pipeline2d (16384^2 bands host to host, 200 steps), "
                         "batched, fp64 (2^20 fp64, 100 steps), 2d (16384^2, "
                         "200 steps, 16 bands), adjoint (8192^2, 100 steps), copy (a one-pass "
                         "1 GiB device copy: the copy ceiling and the counter calibration), "
                         "overhead (the partition benchmark of 2^21..2^28 "
                         "doubles with a runtime-compiled kernel, hx futures against raw HIP "
                         "streams), cpu; 'none' runs the headline only")
    ap.add_argument("--overhead-only", choices=("e1", "e2"), default=None,
                    help="run only one of the paper's overhead experiments and print its JSON "
                         "(the default run starts each in a child process of its own)")
    args = ap.parse_args()
    legs = set(args.legs.split(","))
    if args.overhead_only:
        import paper_1810_11482_amd as hx
        print(json.dumps(overhead_leg(hx, args.overhead_only)), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1810_11482_amd as hx

    n = 1 << args.log2n
    T, r = 50, 0.25
    ctx = hx.hx_ctx_create(0, compute_streams=args.streams, timing=True)
    info = hx.hx_device_info(0)
    log(f"device {info.arch.decode()} CUs={info.compute_units}")
    P = Partitioned(hx, ctx, n, args.parts, T, r)
    tb = T

    # ------------------------------------------- form / geometry sweep (untimed)
    # halos of 52 cells: the 50 the pass reaches, rounded up to whole 16-byte
    # vectors as the propagator form needs (the direct form reads its 50)
    hw = 4 * ((tb + 3) // 4)
    cands = []
    if args.form in ("auto", "direct"):
        cands += [("direct", c, 0) for c in ([args.cells_per_lane] if args.cells_per_lane
                                            else [32, 16])]
    if args.form in ("auto", "propagator"):
        # the block walk (-2, the plan's choice for equal partitions), the
        # interleaved walk and contiguous spans of 128 blocks per wave
        cands += [("propagator", 0, sp) for sp in ([args.span_blocks] if args.span_blocks
                                                  else [-2, -1, 128])]
    swept = []
    for form, cpl_c, span_c in cands:
        fcode = hx.HX_FORM_PROPAGATOR if form == "propagator" else hx.HX_FORM_DIRECT
        bp = BatchedPass(hx, ctx, P, tb, cpl_c or 16, fcode, span_c, hw)
        bp.run(2)
        P.wait()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bp.run(3)
        P.wait()
        t = (time.perf_counter() - t0) / 3
        hx.hx_event_release(ctx, P.last)
        P.last = 0
        bp.close()
        swept.append((t, form, cpl_c or 16, span_c))
        log(f"sweep batched pass form={form} cpl={cpl_c} span={span_c}: {t * 1e3:.3f} ms/step")
    # the project's autotuner decides the timed configuration: pass depth,
    # form, walk or tile geometry (the sweep above only reports the forms)
    tsegs = []
    for p in range(P.parts):
        lp, rp = (p - 1) % P.parts, (p + 1) % P.parts
        tsegs.append(hx.segment(inp=P.A[p], out=P.B[p], n=P.sizes[p], r=r,
                                bc_lo=hx.HX_BC_GHOST, bc_hi=hx.HX_BC_GHOST, halo_lo=P.A[lp],
                                halo_lo_offset=(P.sizes[lp] - hw) * 4, halo_hi=P.A[rp],
                                halo_width=hw))
    if args.form == "auto" and not args.span_blocks and not args.cells_per_lane:
        t0 = time.perf_counter()
        tb_ = hx.hx_tune_batched(ctx, hx.HX_F32, T, tsegs, 4000)
        tuned = {"tuner": "hx_tune_batched", "seconds": time.perf_counter() - t0,
                 "depth": tb_.steps, "passes": T // tb_.steps,
                 "form": "propagator" if tb_.form == hx.HX_FORM_PROPAGATOR else "direct",
                 "span_blocks": tb_.span_blocks, "cells_per_lane": tb_.cells_per_lane,
                 "waves_per_group": tb_.waves_per_group,
                 "grid_waves_per_cu": tb_.grid_waves_per_cu}
        form, tb = tuned["form"], tb_.steps
        cpl = tb_.cells_per_lane or 16
        span = tb_.span_blocks if form == "propagator" else 0
        t_wpg, t_grid = tb_.waves_per_group, tb_.grid_waves_per_cu or -1
        log(f"tuner: {tuned}")
    else:
        _, form, cpl, span = min(swept)
        tuned, t_wpg, t_grid = None, 0, -1
    fcode = hx.HX_FORM_PROPAGATOR if form == "propagator" else hx.HX_FORM_DIRECT
    if span == 0 and form == "propagator":
        span = -2  # the plan's own choice for equal partitions: the block walk
    by_form = {}
    for t, f, c_, s_ in swept:
        key = (f"{f}_cpl{c_}" if f == "direct" else f"{f}_interleaved" if s_ == -1 else
               f"{f}_block_walk" if s_ == -2 else f"{f}_span{s_ or 'auto'}")
        by_form[key] = t * 1e3

    # ------------------------------------------------------------ timed region
    P.reset()
    bp = BatchedPass(hx, ctx, P, tb, cpl, fcode, span, hw, t_wpg, t_grid)
    bp.run(args.warmup)
    if P.last:
        P.wait()
    torch.cuda.synchronize()
    launches = []
    t0 = time.perf_counter()
    bp.run(args.steps, keep=launches)
    P.wait()
    torch.cuda.synchronize()
    sec = (time.perf_counter() - t0) / args.steps
    durs = []
    for e in launches:
        a, b = hx.hx_event_span(ctx, e, e)
        durs.append(b - a)
    for e in launches[:-1]:
        hx.hx_event_release(ctx, e)
    bp.close()
    log("timed launches, ms: " + " ".join(f"{d:.4f}" for d in durs))
    avg_ms = float(np.mean(durs))
    ms_per_step = sec * 1e3
    value = float(n) * T / sec
    # one pass from the initial state, every cell against the oracle (the same
    # serial FP64 run the CPU baseline times)
    P.reset()
    bp = BatchedPass(hx, ctx, P, tb, cpl, fcode, span, hw, t_wpg, t_grid)
    bp.run(1)
    P.wait()
    bp.close()
    cur = P.current()
    got = np.empty(n, np.float32)
    evs = [hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, got[o:].ctypes.data, b, 0, 0, 0,
                                                 s_ * 4), [P.last])
           for (o, s_), b in zip(P.bounds, cur)]
    for e in evs:
        assert hx.hx_wait(ctx, e) == hx.HX_OK
        hx.hx_event_release(ctx, e)
    import oracle
    u0 = np.asarray(P.u0, dtype=np.float64)
    t_or = time.perf_counter()
    ref = oracle.heat1d_periodic(u0, r, T)
    t_or = time.perf_counter() - t_or
    del u0
    g64 = got.astype(np.float64)
    full_err = {"rel_l2": float(np.linalg.norm(g64 - ref) / np.linalg.norm(ref)),
                "max_rel_per_cell": float(np.max(np.abs(g64 - ref) / np.abs(ref))),
                "cells": n}
    del g64, got
    log(f"one pass against the oracle, every cell: {full_err} (oracle {t_or:.2f} s)")

    cells_per_launch = float(n)
    bytes_per_launch = cells_per_launch * BYTES_PER_CELL_PASS
    bw = bytes_per_launch / (avg_ms * 1e-3)
    hbm_frac = bw / HBM_PEAK
    fp16_walk = form == "propagator" and span in (-1, -2)
    kform = ({-1: "propagator_il", -2: "propagator_bw"}.get(span, form) if form == "propagator"
             else form)
    traffic = measured_traffic(kform)
    if form == "propagator":
        # matrix-core work, unpruned: 1024-cell blocks x NC window chunks x
        # six 32x32x16 bf16 products (span walk) or three fp16 ones (block and
        # interleaved walks); NC = 9 at 50 steps
        od = 8 * ((tb + 7) // 8)
        nc = (32 + tb + od + 15) // 16
        mf_per_launch = cells_per_launch / 1024 * nc * (MFMA_FLOPS_PER_CHUNK_IL if fp16_walk
                                                        else MFMA_FLOPS_PER_CHUNK)
        mf = mf_per_launch / (avg_ms * 1e-3)
        mfma_frac = mf / MFMA_16BIT_PEAK
        kname = {-1: f"k_prop1d_il<{nc}>", -2: f"k_prop1d_bw<{nc}>"}.get(span, f"k_prop1d<{nc}>")
        if mfma_frac >= hbm_frac:
            roof = {"bound": "mfma", "achieved": mf / 1e12, "peak": MFMA_16BIT_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": mfma_frac}
        else:
            roof = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9,
                    "unit": "GB/s", "frac": hbm_frac}
        mkey = "mfma_fp16_flops_per_launch" if fp16_walk else "mfma_bf16_flops_per_launch"
        roof.update({mkey: mf_per_launch, "mfma_frac": mfma_frac})
    else:
        flops_per_launch = cells_per_launch * tb * FLOPS_PER_UPDATE_1D
        fl = flops_per_launch / (avg_ms * 1e-3)
        alu_frac = fl / VALU_F32_PEAK
        kname = f"k_stencil1d_flat<float,{cpl}>"
        if alu_frac >= hbm_frac:
            roof = {"bound": "alu", "achieved": fl / 1e12, "peak": VALU_F32_PEAK / 1e12,
                    "unit": "TFLOP/s", "frac": alu_frac}
        else:
            roof = {"bound": "hbm", "achieved": bw / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
                    "frac": hbm_frac}
        roof.update({"algorithmic_flops_per_launch": flops_per_launch, "alu_frac": alu_frac})
    roof.update({"traffic": traffic, "kernel": kname, "avg_launch_ms": avg_ms,
                 "launches": len(durs), "algorithmic_bytes_per_launch": bytes_per_launch,
                 "hbm_algorithmic_GBps": bw / 1e9, "hbm_frac": hbm_frac,
                 "kernel_source_hash": kernel_source_hash(kform)})
    log(f"headline ({form}): {ms_per_step:.3f} ms/step, {value:.4e} cell-updates/s, kernel avg "
        f"{avg_ms:.4f} ms")
    check = ("; every 1024-cell block checks its outputs against the split's and the "
             "pruning's absolute error bound and is stepped in f32 by its own wave, in the "
             "same launch, when an output is non-finite or too small for that bound")
    if fp16_walk:
        walk = ("block walk (one wave per 1024-cell block, the tap operands staged in LDS "
                "from a table the plan builds)" if span == -2 else
                "interleaved walk (a persistent grid)")
        form_desc = (f"propagator, {walk}: the 50 steps as one convolution with the "
                     "50-step propagator (101 taps, FP64 on the host), a banded Toeplitz product "
                     "on 32x32x16 fp16 matrix-core tiles; each 1152-cell window scaled by a "
                     "power of two and split into two fp16 terms (hi + lo), the taps likewise, "
                     "three products per pair (hi*hi, hi*lo, lo*hi) accumulated in f32" + check)
    elif form == "propagator":
        form_desc = ("propagator, span walk: the 50 steps as one convolution with the 50-step "
                     "propagator (101 taps, FP64 on the host), a banded Toeplitz product on "
                     "32x32x16 bf16 matrix-core tiles; every f32 operand split exactly into "
                     "three bf16 terms, six products per pair accumulated in f32" + check)
    else:
        form_desc = ("direct: the tile kernel advancing the 50 steps in registers on the vector "
                     "ALUs (no matrix cores)")
    # the form without the matrix cores, from the sweep
    direct_ms = min((v for k_, v in by_form.items() if k_.startswith("direct")), default=None)
    no_mfma = None if direct_ms is None else {
        "form": "direct (vector ALUs only)", "ms_per_step": direct_ms,
        "cell_updates_per_s": float(n) * T / (direct_ms * 1e-3),
        "hbm_algorithmic_frac": float(n) * BYTES_PER_CELL_PASS / (direct_ms * 1e-3) / HBM_PEAK,
        "note": "host wall time per 50-step run in the untimed sweep"}

    result = {
        "metric": "stencil cell-updates/s + HBM GB/s vs roofline; % copy hidden; batched vs plain",
        "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"1D periodic heat stencil, 2^{args.log2n} fp32 cells in "
                               f"{args.parts} partitions of 4 Mi cells, r=0.25, 50 steps, "
                               f"seeded U[0,1] input, with the partitions resident in HBM (one "
                               f"arena): a future graph of one batched launch over all "
                               f"partitions per {tb}-step pass, halos read from neighbour "
                               f"partitions; the same configuration host to host (pinned "
                               f"partitions, H2D -> kernel -> D2H overlapped) is host_to_host",
                   "cells": n, "parts": args.parts, "time_steps": T, "time_block": tb,
                   "update_form": form_desc,
                   "cells_per_lane": cpl if form == "direct" else None,
                   "span_blocks": ({-1: "interleaved walk", -2: "block walk"}.get(
                       span, span or "plan's choice") if form == "propagator" else None),
                   "halo_width": hw, "launches_per_step": bp.passes,
                   "error_vs_oracle_every_cell": full_err},
        "roofline": roof,
        "tuned": tuned,
        "pass_ms_by_form": by_form,
        "no_mfma": no_mfma,
    }
    hx.hx_event_release(ctx, P.last)
    P.last = 0

    # --------------------------------------------------------------- side legs
    if "graph" in legs:
        result["graph_per_partition"] = graph_leg(hx, ctx, P, T, r)
    if "plain" in legs:
        # plain comparator: one launch per partition per step, Algorithm 1 order
        P.reset()
        time_steps(P, 1, hx.HX_PART_PLAIN, 1, 8)
        t_plain, _ = time_steps(P, 1, hx.HX_PART_PLAIN, 1, 8)
        result["plain"] = {"ms_per_step": t_plain * 1e3, "launches_per_step": args.parts * T,
                           "speedup_headline_vs_plain": t_plain / sec}
        log(f"plain: {t_plain * 1e3:.3f} ms/step")
        hx.hx_event_release(ctx, P.last)
        P.last = 0
        result["plain"].update(plain_graph_leg(hx, ctx, P, T, r))
    result["host_to_host"] = pipeline_leg(hx, ctx, P, T, r, cpl, ref)
    del ref
    result["host_link"] = host_link_leg(hx, P)
    # the floor any overlap can reach host to host: every byte over the link
    # in both directions at once (1 GiB each way at the link's two-way rate)
    floor = result["host_link"]["both"]["ms"]
    result["host_to_host"]["host_link_floor_ms"] = floor
    result["host_to_host"]["wall_over_floor"] = result["host_to_host"]["wall_ms"] / floor
    result["host_to_host"]["copies_alone_over_floor"] = \
        result["host_to_host"]["copies_alone_ms"] / floor
    if "pipeline2d" in legs:
        result["pipeline_2d"] = pipeline2d_leg(hx)
    if "copy" in legs:
        result["copy_calibration"] = copy_leg(hx, ctx, P)
    if "batched" in legs:
        result["batched"] = batched_leg(hx, ctx)
    if "fp64" in legs:
        result["periodic_fp64"] = fp64_leg(hx, ctx)
    if "2d" in legs:
        result["banded_2d"] = banded2d_leg(hx, ctx)
    if "adjoint" in legs:
        result["adjoint"] = adjoint_leg(hx, ctx)
    if "overhead" in legs:
        result["overhead_vs_native"] = overhead_in_child()

    # --------------------------------------------------------------- CPU oracle
    if "cpu" in legs:
        result["cpu_baseline"] = cpu_baseline(n * T / t_or, t_or, n, T)
        result["oracle_timings"] = oracle_timings()

    print(json.dumps(result), flush=True)
    hx.hx_ctx_destroy(ctx)


def graph_leg(hx, ctx, P, T, r):
    """The per-partition future graph: node (p, b) advances partition p by one
    time block and depends on (p-1, b-1), (p, b-1), (p+1, b-1); nodes spread
    over the context's compute streams and run concurrently."""
    best = None
    for tb, cpl in ((50, 32), (50, 16), (25, 32)):
        P.reset()
        time_steps(P, 2, hx.HX_PART_GRAPH, tb, cpl)
        sec, nodes = time_steps(P, 5, hx.HX_PART_GRAPH, tb, cpl, nodes=True)
        durs = []
        for e in nodes:
            a, b = hx.hx_event_span(ctx, e, e)
            durs.append(b - a)
            hx.hx_event_release(ctx, e)
        log(f"per-partition graph tb={tb} cpl={cpl}: {sec * 1e3:.3f} ms/step, node avg "
            f"{np.mean(durs) * 1e3:.1f} us")
        cand = {"ms_per_step": sec * 1e3, "cell_updates_per_s": P.n * T / sec, "time_block": tb,
                "cells_per_lane": cpl, "launches_per_step": P.parts * -(-T // tb),
                "node_avg_ms": float(np.mean(durs)),
                "kernel_concurrency": float(np.sum(durs)) / (sec * 1e3 * 5)}
        if best is None or cand["ms_per_step"] < best["ms_per_step"]:
            best = cand
    hx.hx_event_release(ctx, P.last)
    P.last = 0
    return best


def batched_leg(hx, ctx, reps=5):
    """4096 independent periodic problems (sizes log-uniform in [1024, 2^20], r
    in [0.05, 0.25], 20 steps, fp32): persistent launch, captured graph and the
    plain one-launch-per-problem-per-step form."""
    import torch
    import oracle
    import workloads
    spec = workloads.Batched1D()
    sizes, rs, offs = workloads.batched1d_problems(spec)
    total = int(sizes.sum())
    u0 = workloads.batched1d_u0(spec)
    bufs = [hx.hx_buffer_create(ctx, total * 4) for _ in range(3)]
    ev = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, u0.ctypes.data, bufs[0], 0, 0, 0,
                                               total * 4))
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    hx.hx_event_release(ctx, ev)
    segs = [hx.segment(inp=bufs[0], in_offset=int(o) * 4, out=bufs[1], out_offset=int(o) * 4,
                       tmp=bufs[2], tmp_offset=int(o) * 4, n=int(n), r=float(rr),
                       bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
            for o, n, rr in zip(offs, sizes, rs)]
    updates = float(total) * spec.steps
    res = {"problems": spec.count, "cells": total, "steps": spec.steps}

    def timed(plan, n):
        e = hx.hx_launch_batched(ctx, plan)
        assert hx.hx_wait(ctx, e) == hx.HX_OK, hx.hx_last_error(ctx)
        hx.hx_event_release(ctx, e)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs = []
        for _ in range(n):  # chained, so the launches run one after another
            evs.append(hx.hx_launch_batched(ctx, plan, deps=evs[-1:]))
        assert hx.hx_wait(ctx, evs[-1]) == hx.HX_OK
        sec = (time.perf_counter() - t0) / n
        for e in evs:
            hx.hx_event_release(ctx, e)
        return sec

    # the project's autotuner picks the pass depth (20 steps in one pass, or
    # several passes ping-ponging between two buffers), the form and the tile
    # geometry, timing each candidate on the GPU
    t0 = time.perf_counter()
    tb_ = hx.hx_tune_batched(ctx, hx.HX_F32, spec.steps, segs, 4000)
    tune_s = time.perf_counter() - t0
    D = tb_.steps
    passes = spec.steps // D
    kw = dict(cells_per_lane=tb_.cells_per_lane, waves_per_group=tb_.waves_per_group,
              grid_waves_per_cu=tb_.grid_waves_per_cu, form=tb_.form,
              span_blocks=tb_.span_blocks)
    plans = [hx.hx_plan_create_batched(ctx, hx.HX_F32, D, segs, hx.HX_BATCH_PERSISTENT, **kw)]
    if passes > 1:  # the return pass: out -> in
        back = [hx.segment(inp=bufs[1], in_offset=int(o) * 4, out=bufs[0],
                           out_offset=int(o) * 4, n=int(n), r=float(rr),
                           bc_lo=hx.HX_BC_PERIODIC, bc_hi=hx.HX_BC_PERIODIC)
                for o, n, rr in zip(offs, sizes, rs)]
        plans.append(hx.hx_plan_create_batched(ctx, hx.HX_F32, D, back, hx.HX_BATCH_PERSISTENT,
                                               **kw))

    def run_tuned(n_runs):
        """n_runs whole 20-step runs, chained; returns the last event."""
        last = 0
        for _ in range(n_runs):
            for k in range(passes):
                e = hx.hx_launch_batched(ctx, plans[k % 2], deps=[last] if last else [])
                if last:
                    hx.hx_event_release(ctx, last)
                last = e
        return last

    e = run_tuned(1)
    assert hx.hx_wait(ctx, e) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, e)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e = run_tuned(reps)
    assert hx.hx_wait(ctx, e) == hx.HX_OK, hx.hx_last_error(ctx)
    hx.hx_event_release(ctx, e)
    sec = (time.perf_counter() - t0) / reps
    tuned = {"tuner": "hx_tune_batched", "tuner_seconds": tune_s, "depth": D, "passes": passes,
             "form": "propagator" if tb_.form == hx.HX_FORM_PROPAGATOR else "direct",
             "cells_per_lane": tb_.cells_per_lane, "waves_per_group": tb_.waves_per_group,
             "grid_waves_per_cu": tb_.grid_waves_per_cu, "span_blocks": tb_.span_blocks}
    log(f"batched persistent, tuned {tuned}: {sec * 1e3:.3f} ms")
    res["persistent"] = {"ms": sec * 1e3, "cell_updates_per_s": updates / sec,
                         "hbm_algorithmic_GBps": total * 8 * passes / sec / 1e9,
                         "hbm_algorithmic_frac": total * 8 * passes / sec / HBM_PEAK,
                         "tuned": tuned}
    # the run's result for the check below: in bufs[1] after an odd number of
    # passes, else in bufs[0]; one run from the initial state
    ev = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, u0.ctypes.data, bufs[0], 0, 0, 0,
                                               total * 4))
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    hx.hx_event_release(ctx, ev)
    e = run_tuned(1)
    assert hx.hx_wait(ctx, e) == hx.HX_OK
    hx.hx_event_release(ctx, e)
    result_buf = bufs[1] if passes % 2 == 1 else bufs[0]
    for pl in plans:
        hx.hx_plan_destroy(ctx, pl)
    # sampled correctness of the persistent result
    rng = np.random.default_rng(9)
    errs = []
    for k in rng.choice(spec.count, 16, replace=False):
        o, n = int(offs[k]), int(sizes[k])
        i = int(rng.integers(0, n))
        got = np.empty(1, np.float32)
        e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, got.ctypes.data, result_buf,
                                                  (o + i) * 4, 0, 0, 4))
        assert hx.hx_wait(ctx, e) == hx.HX_OK
        hx.hx_event_release(ctx, e)
        ref = oracle.heat1d_periodic_at(u0[o:o + n].astype(np.float64), float(rs[k]),
                                        spec.steps, [i])[0]
        errs.append(abs(got[0] - ref) / abs(ref))
    res["persistent"]["sampled_max_rel_err"] = float(max(errs))
    ev = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, u0.ctypes.data, bufs[0], 0, 0, 0,
                                               total * 4))
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    hx.hx_event_release(ctx, ev)
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, spec.steps, segs, hx.HX_BATCH_GRAPH,
                                     cells_per_lane=16)
    sec = timed(plan, reps)
    hx.hx_plan_destroy(ctx, plan)
    res["graph"] = {"ms": sec * 1e3, "cell_updates_per_s": updates / sec}
    plan = hx.hx_plan_create_batched(ctx, hx.HX_F32, spec.steps, segs, hx.HX_BATCH_PLAIN,
                                     cells_per_lane=16)
    sec = timed(plan, 1)
    hx.hx_plan_destroy(ctx, plan)
    res["plain"] = {"ms": sec * 1e3, "cell_updates_per_s": updates / sec,
                    "launches": spec.count * spec.steps}
    res["speedup_persistent_vs_plain"] = res["plain"]["ms"] / res["persistent"]["ms"]
    res["speedup_graph_vs_plain"] = res["plain"]["ms"] / res["graph"]["ms"]
    for b in bufs:
        hx.hx_buffer_destroy(ctx, b)
    log(f"batched: {res}")
    return res


def pipeline_leg(hx, ctx0, P, T, r, cpl, ref):
    """The headline configuration host to host: the pinned 2^28-cell input is
    copied in partition by partition, each partition's 50-step kernel waits for
    its own and its neighbours' copies, and its copy out for its kernel
    (hx_run_pipeline), on a context whose default stream set leaves each copy
    stream a hardware queue.  Full runs and copies-only runs (the same graph
    with zero-step kernels, i.e. 16 MiB device copies) alternate, because the
    host link's rate drifts by a few percent between runs; every time is a
    median of nine after a warm-up.  ref: the oracle's result (FP64), against
    which every cell of the host output is checked."""
    import torch
    ctx = hx.hx_ctx_create(0, timing=True)
    P.wait()
    saved = (P.ctx, P.A, P.B, P.last)
    P.ctx = ctx
    P.A = [hx.hx_buffer_create(ctx, s * 4) for s in P.sizes]
    P.B = [hx.hx_buffer_create(ctx, s * 4) for s in P.sizes]
    P.last = 0
    base = hx.partitioned_desc(hx.HX_F32, P.sizes, P.A, P.B, T, r, periodic=True,
                               time_block=T, cells_per_lane=cpl)
    pd = hx.hx_pipeline_desc(base, P.host_in, P.host_out)
    pd0 = hx.hx_pipeline_desc(hx.partitioned_desc(hx.HX_F32, P.sizes, P.A, P.B, 0, r,
                                                  periodic=True, cells_per_lane=cpl),
                              P.host_in, P.host_out)

    def once(desc, spans=False):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev, h2d, ker, d2h = hx.hx_run_pipeline(ctx, desc, op_events=spans)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        w = time.perf_counter() - t0
        sp = None
        if spans:
            ref = h2d[0]
            sp = {"h2d": [hx.hx_event_span(ctx, e, ref) for e in h2d],
                  "kernel": [hx.hx_event_span(ctx, e, ref) for e in ker],
                  "d2h": [hx.hx_event_span(ctx, e, ref) for e in d2h]}
            for e in h2d + ker + d2h:
                hx.hx_event_release(ctx, e)
        hx.hx_event_release(ctx, ev)
        return w, sp

    walls, cw = [], []
    for it in range(10):
        walls.append(once(pd)[0])
        cw.append(once(pd0)[0])
    W, t_copy = float(np.median(walls[1:])), float(np.median(cw[1:]))
    # the timeline of one more full run, and its output: every cell against the
    # oracle
    w_last, spans = once(pd, spans=True)
    out = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * P.n).from_address(P.host_out))
    o64 = out.astype(np.float64)
    err = {"rel_l2": float(np.linalg.norm(o64 - ref) / np.linalg.norm(ref)),
           "max_rel_per_cell": float(np.max(np.abs(o64 - ref) / np.abs(ref))), "cells": P.n}
    del o64
    # kernels alone: the single-pass device-resident graph
    P.cur_in_a = True
    t_kernel, _ = time_steps(P, 3, hx.HX_PART_GRAPH, T, cpl)
    C = intervals_union([tuple(x) for x in spans["h2d"] + spans["d2h"]])
    K = intervals_union([tuple(x) for x in spans["kernel"]])
    CK = intersect_len(C, K)
    eta = (t_copy + t_kernel - W) / min(t_copy, t_kernel)
    bytes_copied = 2 * P.n * 4
    P.wait()
    if P.last:
        hx.hx_event_release(ctx, P.last)
    hx.hx_ctx_destroy(ctx)
    P.ctx, P.A, P.B, P.last = saved
    P.cur_in_a = True
    res = {"value": P.n * T / W, "unit": "cell-updates/s (PCIe-inclusive, host to host)",
           "wall_ms": W * 1e3, "copies_alone_ms": t_copy * 1e3,
           "kernels_alone_ms": t_kernel * 1e3,
           "wall_over_copies_alone": W / t_copy,
           "copy_hidden_literal": CK / measure_len(C),
           "copy_hidden_literal_bound": min(1.0, measure_len(K) / measure_len(C)),
           "kernel_time_under_copies": CK / measure_len(K),
           "overlap_efficiency_eta": eta,
           "host_link_GBps_during_overlap": bytes_copied / (measure_len(C) * 1e-3) / 1e9,
           "host_link_GBps_whole_run": bytes_copied / W / 1e9,
           "error_vs_oracle_every_cell": err,
           "timeline_run_ms": w_last * 1e3,
           "method": "wall times: host clock around each run, medians of 9 (full and "
                     "copies-only runs alternating); spans: HIP events of every copy and kernel "
                     "of the last run (timing context)"}
    log(f"host to host: {res}")
    return res


def host_link_leg(hx, P, reps=7):
    """The host link alone: 1 GiB host to device, 1 GiB device to host, and
    both at once, each as 64 copies of 16 MiB between the pinned arrays and
    device buffers on the context's copy streams (medians of `reps` after a
    warm-up)."""
    import torch
    ctx = hx.hx_ctx_create(0, timing=True)
    A = [hx.hx_buffer_create(ctx, s * 4) for s in P.sizes]
    B = [hx.hx_buffer_create(ctx, s * 4) for s in P.sizes]

    def run(h2d, d2h):
        evs = []
        for (o, s_), a, b in zip(P.bounds, A, B):
            if h2d:
                evs.append(hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, P.host_in + o * 4,
                                                                 a, 0, 0, 0, s_ * 4)))
            if d2h:
                evs.append(hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, P.host_out + o * 4,
                                                                 b, 0, 0, 0, s_ * 4)))
        torch.cuda.synchronize()
        w = hx.hx_when_all(ctx, evs)
        assert hx.hx_wait(ctx, w) == hx.HX_OK, hx.hx_last_error(ctx)
        spans = [hx.hx_event_span(ctx, e, evs[0]) for e in evs]
        for e in evs + [w]:
            hx.hx_event_release(ctx, e)
        return max(b_ for _, b_ in spans) - min(a_ for a_, _ in spans)

    res = {}
    nbytes = P.n * 4
    for key, h, d in (("h2d_alone", True, False), ("d2h_alone", False, True),
                      ("both", True, True)):
        ms = float(np.median([run(h, d) for _ in range(reps + 1)][1:]))
        moved = nbytes * (2 if key == "both" else 1)
        res[key] = {"ms": ms, "GBps": moved / (ms * 1e-3) / 1e9}
    for b in A + B:
        hx.hx_buffer_destroy(ctx, b)
    hx.hx_ctx_destroy(ctx)
    res["method"] = ("HIP events of the copies (first start to last end), 64 x 16 MiB per "
                     "direction, pinned host memory from hx_host_alloc")
    log(f"host link: {res}")
    return res


def pipeline2d_leg(hx):
    """Host-to-host 2D run: 16384^2 fp32, zero-Dirichlet, r = 0.2, 200 steps, 16
    row bands, each copied in, advanced on its extended rows (own rows plus the
    200-row light cone from each neighbour, by device copies) and copied out,
    so that copies of some bands overlap the kernels of others; the overlap
    measures as in the 1D pipeline."""
    import torch
    import oracle
    import workloads
    from paper_1810_11482_amd.pipeline2d import Pipeline2D
    spec = workloads.Banded2D()
    u0 = workloads.banded2d_u0(spec)
    ny, nx, T, r = spec.ny, spec.nx, spec.steps, spec.r
    cells = ny * nx
    ctx = hx.hx_ctx_create(0, timing=True)
    hin = hx.hx_host_alloc(ctx, cells * 4)
    hout = hx.hx_host_alloc(ctx, cells * 4)
    np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * cells).from_address(hin))[:] = \
        u0.ravel()
    out = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_float * cells).from_address(hout))
    hx_ctx = ctx
    # 64 rows per wave: two bands' kernels share the GPU at a time here
    pl = Pipeline2D(ctx, ny, nx, workloads.band_bounds(ny, spec.bands), T, r, time_block=16,
                    cells_per_lane=4, rows_per_block=64)

    def timed(fn, reps=3):
        """Wall time of fn() to its final event: the mean after the first of
        `reps` runs (the only run when reps is 1); returns it and the last
        run's events (earlier runs' are released)."""
        walls, last = [], None
        for it in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            assert hx.hx_wait(hx_ctx, res[0]) == hx.HX_OK, hx.hx_last_error(hx_ctx)
            walls.append(time.perf_counter() - t0)
            if last:
                for e in [x for grp in last for x in (grp if isinstance(grp, list) else [grp])]:
                    hx.hx_event_release(hx_ctx, e)
            last = res
        return float(np.mean(walls[1:] if reps > 1 else walls)), last

    # the host link's rate drifts between runs: full runs and copies-only runs
    # alternate, and each time is the median of five after a warm-up
    walls, cwalls, res = [], [], None
    for it in range(6):
        w_, res_ = timed(lambda: pl.run(hin, hout), reps=1)
        if res:
            for e in [res[0]] + res[1] + res[2] + res[3]:
                hx.hx_event_release(ctx, e)
        res = res_
        walls.append(w_)
        c_, cres = timed(lambda: pl.run(hin, hout, kernels=False), reps=1)
        for e in [cres[0]] + cres[1] + cres[3]:
            hx.hx_event_release(ctx, e)
        cwalls.append(c_)
    W, t_copy = float(np.median(walls[1:])), float(np.median(cwalls[1:]))
    # the last full run's output and spans
    w_, res_ = timed(lambda: pl.run(hin, hout), reps=1)
    for e in [res[0]] + res[1] + res[2] + res[3]:
        hx.hx_event_release(ctx, e)
    res = res_
    _, h2d, ker, d2h = res
    ref0 = h2d[0]
    spans = {"h2d": [hx.hx_event_span(ctx, e, ref0) for e in h2d],
             "kernel": [hx.hx_event_span(ctx, e, ref0) for e in ker],
             "d2h": [hx.hx_event_span(ctx, e, ref0) for e in d2h]}
    for e in [res[0]] + h2d + ker + d2h:
        hx.hx_event_release(ctx, e)
    # sampled correctness before anything else touches host_out
    rng = np.random.default_rng(14)
    pts = [(0, 0), (1023, 5000), (1024, 5000), (ny - 1, nx - 1)] + \
        [(int(a), int(b)) for a, b in zip(rng.integers(0, ny, 6), rng.integers(0, nx, 6))]
    ref = oracle.heat2d_dirichlet_at(u0, r, T, pts)
    got = np.array([out[y * nx + x] for y, x in pts], dtype=np.float64)
    err = float(np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)))
    t_kernel, res = timed(lambda: pl.kernels_only())
    for e in [res[0]] + res[1]:
        hx.hx_event_release(ctx, e)
    C = intervals_union([tuple(x) for x in spans["h2d"] + spans["d2h"]])
    K = intervals_union([tuple(x) for x in spans["kernel"]])
    lit = intersect_len(C, K) / measure_len(C)
    eta = (t_copy + t_kernel - W) / min(t_copy, t_kernel)
    ext = sum(pl.ext_rows) / ny
    pl.close()
    hx.hx_host_free(ctx, hin)
    hx.hx_host_free(ctx, hout)
    hx.hx_ctx_destroy(ctx)
    res = {"ny": ny, "nx": nx, "bands": spec.bands, "steps": T,
           "wall_ms": W * 1e3, "copies_alone_ms": t_copy * 1e3, "kernels_alone_ms": t_kernel * 1e3,
           "pcie_inclusive_cell_updates_per_s": cells * T / W,
           "recomputed_rows_factor": ext,
           "copy_hidden_literal": lit, "overlap_efficiency_eta": eta,
           "copy_bound_efficiency": t_copy / W,
           "host_link_GBps_during_overlap": 2 * cells * 4 / (measure_len(C) * 1e-3) / 1e9,
           "sampled_max_rel_err": err}
    log(f"pipeline 2D: {res}")
    return res


def fp64_leg(hx, ctx, reps=10):
    """2^20 fp64 periodic cells, r = 0.25, 100 steps in one fused launch (the
    sine-mode workload); checked against the FP64 oracle."""
    import oracle
    import workloads
    spec = workloads.Periodic1D()
    u0 = workloads.periodic1d_u0(spec)
    n = spec.n
    a = hx.hx_buffer_create(ctx, n * 8)
    b = hx.hx_buffer_create(ctx, n * 8)
    e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, u0.ctypes.data, a, 0, 0, 0, n * 8))
    assert hx.hx_wait(ctx, e) == hx.HX_OK
    hx.hx_event_release(ctx, e)
    best = None
    for cpl, tb in ((32, 100), (16, 100), (64, 100), (32, 50)):
        args = hx.stencil_args(dims=1, dtype=hx.HX_F64, nx=n, steps=spec.steps, r=spec.r, inp=a,
                               out=b, tmp=hx.hx_buffer_create(ctx, n * 8) if tb < 100 else 0,
                               cells_per_lane=cpl, time_block=tb)
        evs = [hx.hx_launch_stencil(ctx, args) for _ in range(reps + 1)]
        assert hx.hx_wait(ctx, evs[-1]) == hx.HX_OK
        d = [y - x for x, y in (hx.hx_event_span(ctx, ev, ev) for ev in evs[1:])]
        for ev in evs:
            hx.hx_event_release(ctx, ev)
        ms = float(np.median(d))
        log(f"fp64 1D cpl={cpl} tb={tb}: {ms * 1e3:.1f} us")
        if best is None or ms < best[0]:
            best = (ms, cpl, tb)
    out = np.empty(n, np.float64)
    e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, out.ctypes.data, b, 0, 0, 0, n * 8))
    assert hx.hx_wait(ctx, e) == hx.HX_OK
    hx.hx_event_release(ctx, e)
    ref = oracle.heat1d_periodic(u0, spec.r, spec.steps)
    err = float(np.linalg.norm(out - ref) / np.linalg.norm(ref))
    return {"cells": n, "steps": spec.steps, "ms": best[0], "cells_per_lane": best[1],
            "time_block": best[2], "cell_updates_per_s": n * spec.steps / (best[0] * 1e-3),
            "rel_l2_vs_oracle": err}


def banded2d_leg(hx, ctx):
    """16384^2 fp32, zero-Dirichlet, r = 0.2, 200 steps, 16 row bands with
    halo-row futures (the per-band future graph), Gaussian-bump field."""
    import torch
    import workloads
    spec = workloads.Banded2D()
    u0 = workloads.banded2d_u0(spec)
    bounds = workloads.band_bounds(spec.ny, spec.bands)
    cells = spec.ny * spec.nx
    arena_a = hx.hx_buffer_create(ctx, cells * 4)
    arena_b = hx.hx_buffer_create(ctx, cells * 4)
    pa, _ = hx.hx_buffer_ptr(ctx, arena_a)
    pb, _ = hx.hx_buffer_ptr(ctx, arena_b)
    row = spec.nx * 4
    A = [hx.hx_buffer_wrap(ctx, pa + o * row, s * row) for o, s in bounds]
    B = [hx.hx_buffer_wrap(ctx, pb + o * row, s * row) for o, s in bounds]

    def upload():
        e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, u0.ctypes.data, arena_a, 0, 0, 0,
                                                  u0.nbytes))
        assert hx.hx_wait(ctx, e) == hx.HX_OK
        hx.hx_event_release(ctx, e)
    # the project's autotuner picks the 2D geometry (time block, columns per
    # lane, rows per wave) on the whole grid as one array, 200 steps, timing
    # each candidate on the GPU; the band graph then runs with it, next to two
    # fixed geometries for comparison
    upload()
    t0 = time.perf_counter()
    arena_t = hx.hx_buffer_create(ctx, cells * 4)
    targs = hx.stencil_args(dims=2, dtype=hx.HX_F32, nx=spec.nx, ny=spec.ny, steps=spec.steps,
                            r=spec.r, inp=arena_a, out=arena_b, tmp=arena_t,
                            bc_lo=hx.HX_BC_DIRICHLET0, bc_hi=hx.HX_BC_DIRICHLET0)
    tbest = hx.hx_tune_stencil(ctx, targs, 4000)
    hx.hx_buffer_destroy(ctx, arena_t)
    tuned = {"tuner": "hx_tune_stencil", "seconds": time.perf_counter() - t0,
             "time_block": tbest.time_block, "cells_per_lane": tbest.cells_per_lane,
             "rows_per_block": tbest.rows_per_block, "waves_per_group": tbest.waves_per_group}
    log(f"2D tuner: {tuned}")
    best = None
    per_mode = {}
    geoms = [(tbest.time_block, tbest.cells_per_lane, tbest.rows_per_block)]
    for g in ((16, 4, 128), (8, 4, 64)):
        if g not in geoms:
            geoms.append(g)
    cands = [(mode, tb, cpl, rows) for mode in (hx.HX_PART_BATCHED, hx.HX_PART_GRAPH)
             for tb, cpl, rows in geoms]
    for mode, tb, cpl, rows in cands:
        upload()
        d = hx.partitioned_desc(hx.HX_F32, [s for _, s in bounds], A, B, spec.steps, spec.r,
                                periodic=False, time_block=tb, cells_per_lane=cpl, dims=2,
                                nx=spec.nx, rows_per_block=rows, mode=mode)
        ts = []
        for it in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ev, in_b, _ = hx.hx_run_partitioned(ctx, d)
            assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
            ts.append(time.perf_counter() - t0)
            hx.hx_event_release(ctx, ev)
        sec = ts[-1]
        mname = "batched" if mode == hx.HX_PART_BATCHED else "graph"
        log(f"2D bands {mname} tb={tb} cpl={cpl} rows={rows}: {sec * 1e3:.2f} ms")
        if best is None or sec < best[0]:
            best = (sec, tb, cpl, rows, mode)
        by_mode = per_mode.setdefault(mname, sec)
        per_mode[mname] = min(by_mode, sec)
    sec, tb, cpl, rows, mode = best
    passes = -(-spec.steps // tb)
    res = {"ny": spec.ny, "nx": spec.nx, "bands": spec.bands, "steps": spec.steps, "ms": sec * 1e3,
           "cell_updates_per_s": cells * spec.steps / sec, "time_block": tb, "cells_per_lane": cpl,
           "rows_per_block": rows,
           "form": "one launch per pass over all bands" if mode == hx.HX_PART_BATCHED
           else "one launch per band per pass",
           "ms_by_form": {k: v * 1e3 for k, v in per_mode.items()},
           "tuned": tuned,
           "hbm_algorithmic_GBps": cells * 8 * passes / sec / 1e9,
           "hbm_algorithmic_frac": cells * 8 * passes / sec / HBM_PEAK}
    # sampled correctness of the best configuration against the oracle
    import oracle
    d = hx.partitioned_desc(hx.HX_F32, [s for _, s in bounds], A, B, spec.steps, spec.r,
                            periodic=False, time_block=tb, cells_per_lane=cpl, dims=2,
                            nx=spec.nx, rows_per_block=rows, mode=mode)
    upload()
    ev, in_b, _ = hx.hx_run_partitioned(ctx, d)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    hx.hx_event_release(ctx, ev)
    rng = np.random.default_rng(13)
    pts = [(0, 0), (1023, 5000), (1024, 5000), (spec.ny - 1, spec.nx - 1)] + \
        [(int(a), int(b)) for a, b in zip(rng.integers(0, spec.ny, 6), rng.integers(0, spec.nx, 6))]
    ref = oracle.heat2d_dirichlet_at(u0, spec.r, spec.steps, pts)
    errs = []
    for (y, x), rv in zip(pts, ref):
        v = np.empty(1, np.float32)
        e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, v.ctypes.data,
                                                  arena_b if in_b else arena_a,
                                                  (y * spec.nx + x) * 4, 0, 0, 4))
        assert hx.hx_wait(ctx, e) == hx.HX_OK
        hx.hx_event_release(ctx, e)
        errs.append(abs(float(v[0]) - rv) / max(abs(rv), 1e-3))
    res["sampled_max_rel_err"] = float(max(errs))
    for b_ in A + B + [arena_a, arena_b]:
        hx.hx_buffer_destroy(ctx, b_)
    return res


def adjoint_leg(hx, ctx):
    """8192^2 fp32 variable-coefficient run, dt = 0.2, 100 steps, S = 10:
    forward with checkpoints, FP64 loss, checkpointed backward."""
    import torch
    import workloads
    spec = workloads.VarCoef2D()
    u0, kappa, y = workloads.varcoef2d_inputs(spec)
    n = spec.ny * spec.nx
    S, nseg = hx.hx_vc_schedule(spec.steps, spec.ckpt)

    def dev(arr=None, nbytes=None):
        b = hx.hx_buffer_create(ctx, arr.nbytes if arr is not None else nbytes)
        if arr is not None:
            e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, arr.ctypes.data, b, 0, 0, 0,
                                                      arr.nbytes))
            assert hx.hx_wait(ctx, e) == hx.HX_OK
            hx.hx_event_release(ctx, e)
        return b
    bu0, bk, by = dev(u0), dev(kappa), dev(y)
    st = n * 4
    buT, bck, bw, bseg = dev(nbytes=st), dev(nbytes=(nseg - 1) * st), dev(nbytes=2 * st),         dev(nbytes=(S - 1) * st)
    blT, bl0, bg64, bga = dev(nbytes=st), dev(nbytes=st), dev(nbytes=n * 8), dev(nbytes=st)
    bloss, work = dev(nbytes=8), dev(nbytes=4096 * 8)
    a = hx.hx_vc_args(hx.HX_F32, spec.nx, spec.ny, spec.dt, spec.steps, spec.ckpt, bu0, bk, buT,
                      bck, bw, bseg, blT, bl0, bg64, bga, 0)
    times = {}
    for it in range(2):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e1 = hx.hx_heat_vc_forward(ctx, a)
        assert hx.hx_wait(ctx, e1) == hx.HX_OK, hx.hx_last_error(ctx)
        t1 = time.perf_counter()
        e2 = hx.hx_launch_loss(ctx, hx.HX_F32, n, buT, by, blT, bloss, work, deps=[e1])
        e3 = hx.hx_heat_vc_backward(ctx, a, deps=[e2])
        assert hx.hx_wait(ctx, e3) == hx.HX_OK, hx.hx_last_error(ctx)
        t2 = time.perf_counter()
        for e in (e1, e2, e3):
            hx.hx_event_release(ctx, e)
        times = {"forward_ms": (t1 - t0) * 1e3, "backward_ms": (t2 - t1) * 1e3}
    T = spec.steps
    # The forward runs each stretch between kept states in fused passes of at
    # most four steps (aligned grids, as here); one pass reads u and kappa and
    # writes u once, whatever its depth.
    fwd_passes = sum(-(-min(S, T - t0) // 4) for t0 in range(0, T, S))
    fwd_bytes = n * fwd_passes * 12   # u read + write, kappa read per pass
    # the backward recomputes each segment's inner states in fused passes
    # that store every level: per pass one read of u and kappa, per state one
    # write
    inner = [min(S, T - t0) - 1 for t0 in range(0, T, S)]
    rec_bytes = n * sum(8 * (-(-m // 4)) + 4 * m for m in inner)
    # the reverse sweep runs in fused passes of up to four adjoint steps: per
    # pass lam, kappa and the accumulator read once and lam and the
    # accumulator written once (20 B), per step its u_t read once (4 B); the
    # segment's first pass does not read the accumulator (-4 B) and its last
    # adds it to the FP64 total instead of storing it (+12 B)
    segs_len = [min(S, T - t0) for t0 in range(0, T, S)]
    adj_bytes = n * sum(20 * (-(-m // 4)) + 4 * m + 8 for m in segs_len)
    res = {"cells": n, "steps": T, "segment": S, **times, "forward_passes": fwd_passes,
           "forward_cell_updates_per_s": n * T / (times["forward_ms"] * 1e-3),
           "forward_hbm_algorithmic_GBps": fwd_bytes / (times["forward_ms"] * 1e-3) / 1e9,
           "backward_hbm_algorithmic_GBps": (rec_bytes + adj_bytes) /
                                            (times["backward_ms"] * 1e-3) / 1e9}
    loss = np.empty(1, np.float64)
    e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, loss.ctypes.data, bloss, 0, 0, 0, 8))
    assert hx.hx_wait(ctx, e) == hx.HX_OK
    hx.hx_event_release(ctx, e)
    res["loss"] = float(loss[0])
    for b_ in (bu0, bk, by, buT, bck, bw, bseg, blT, bl0, bg64, bga, bloss, work):
        hx.hx_buffer_destroy(ctx, b_)
    log(f"adjoint: {res}")
    return res


def plain_chain(hx, ctx, P, T, r, deps=()):
    """The plain form's launches submitted one by one from here: for each of
    the T steps, one one-step launch per partition (halos of one cell read
    from the neighbours' views), every launch after the previous one, as
    HX_PART_PLAIN issues them.  Returns the launch events and where the
    result is (True: the B views)."""
    evs, last = [], list(deps)
    src, dst = P.A, P.B
    for _ in range(T):
        for p in range(P.parts):
            lp, rp = (p - 1) % P.parts, (p + 1) % P.parts
            a = hx.stencil_args(dims=1, dtype=hx.HX_F32, nx=P.sizes[p], steps=1, r=r,
                                inp=src[p], out=dst[p], bc_lo=hx.HX_BC_GHOST,
                                bc_hi=hx.HX_BC_GHOST, halo_lo=src[lp],
                                halo_lo_offset=(P.sizes[lp] - 1) * 4, halo_hi=src[rp],
                                halo_hi_offset=0, halo_width=1, cells_per_lane=8)
            e = hx.hx_launch_stencil(ctx, a, last)
            evs.append(e)
            last = [e]
        src, dst = dst, src
    return evs, T % 2 == 1


def plain_graph_leg(hx, ctx, P, T, r, reps=5):
    """Per-operation cost of the plain form (3200 dependent one-step launches
    per 50-step run): submitted one by one through the futures, against the
    same launches captured once as a graph (hx_graph_begin/end) and replayed
    with one hx_graph_launch.  The captured replay is checked bit for bit
    against the eager run."""
    import torch
    ops = T * P.parts
    # eager, timed on the host, with per-launch spans
    best = None
    for _ in range(2):
        P.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        evs, in_b = plain_chain(hx, ctx, P, T, r)
        t_sub = time.perf_counter() - t0
        assert hx.hx_wait(ctx, evs[-1]) == hx.HX_OK, hx.hx_last_error(ctx)
        t_all = time.perf_counter() - t0
        spans = [b - a for a, b in (hx.hx_event_span(ctx, e, e) for e in evs)]
        for e in evs:
            hx.hx_event_release(ctx, e)
        if best is None or t_all < best[1]:
            best = (t_sub, t_all, float(np.mean(spans)))
    eager_out = np.empty(P.n, np.float32)
    for (o, s_), b in zip(P.bounds, P.B if in_b else P.A):
        eager_out[o:o + s_] = download_f32(hx, ctx, b, s_)
    # the same launches captured once, replayed
    P.reset()
    t0 = time.perf_counter()
    hx.hx_graph_begin(ctx)
    evs, in_b2 = plain_chain(hx, ctx, P, T, r)
    g = hx.hx_graph_end(ctx)
    t_cap = time.perf_counter() - t0
    for e in evs:
        hx.hx_event_release(ctx, e)
    ts = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev = hx.hx_graph_launch(ctx, g)
        assert hx.hx_wait(ctx, ev) == hx.HX_OK, hx.hx_last_error(ctx)
        ts.append(time.perf_counter() - t0)
        hx.hx_event_release(ctx, ev)
    # one replay from the initial state against the eager run
    P.reset()
    ev = hx.hx_graph_launch(ctx, g)
    assert hx.hx_wait(ctx, ev) == hx.HX_OK
    hx.hx_event_release(ctx, ev)
    graph_out = np.empty(P.n, np.float32)
    for (o, s_), b in zip(P.bounds, P.B if in_b2 else P.A):
        graph_out[o:o + s_] = download_f32(hx, ctx, b, s_)
    same = bool(np.array_equal(graph_out, eager_out))
    hx.hx_plan_destroy(ctx, g)
    P.reset()
    t_graph = float(np.median(ts))
    res = {"operations": ops,
           "eager_submit_us_per_op": best[0] / ops * 1e6,
           "eager_us_per_op": best[1] / ops * 1e6,
           "graph_replay_ms_per_step": t_graph * 1e3,
           "graph_replay_us_per_op": t_graph / ops * 1e6,
           "graph_capture_ms": t_cap * 1e3,
           "eager_span_us_per_op": best[2] * 1e3,
           "graph_equals_eager_bitwise": same,
           "method": "host clock around each run (eager: best of 2; replay: median of 5); "
                     "eager span: mean HIP-event span of the eager launches (the kernel plus "
                     "the markers and dispatch between launches; the kernels' own duration "
                     "is in the kernel-trace profile of this leg)"}
    log(f"plain chain: {res}")
    assert same, "the captured plain chain differs from the eager run"
    return res


def download_f32(hx, ctx, buf, n):
    out = np.empty(n, np.float32)
    e = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, out.ctypes.data, buf, 0, 0, 0, n * 4))
    assert hx.hx_wait(ctx, e) == hx.HX_OK
    hx.hx_event_release(ctx, e)
    return out


def copy_leg(hx, ctx, P, reps=5):
    """A one-pass device copy of the whole arena (hx_copy_async D2D: the
    library's vector copy kernel, one 16-byte nontemporal load and store per
    thread, 4 KiB per workgroup): 1 GiB read and 1 GiB written.  It is the
    practical HBM ceiling the stencil kernels are held against, and the kernel
    whose HBM counters scale the stencil's."""
    d = hx.hx_copy_desc(hx.HX_D2D, 0, P.arena_b, 0, P.arena_a, 0, P.n * 4)
    evs = [hx.hx_copy_async(ctx, d)]
    for _ in range(reps):
        evs.append(hx.hx_copy_async(ctx, d, deps=[evs[-1]]))
    assert hx.hx_wait(ctx, evs[-1]) == hx.HX_OK, hx.hx_last_error(ctx)
    dur = [b - s_ for s_, b in (hx.hx_event_span(ctx, e, e) for e in evs)]
    for e in evs:
        hx.hx_event_release(ctx, e)
    ms = float(np.median(dur[1:]))
    nbytes = P.n * 8
    return {"kernel": "k_copy16", "cells": P.n, "bytes_moved": nbytes, "avg_ms": ms,
            "GBps": nbytes / (ms * 1e-3) / 1e9, "frac_of_peak": nbytes / (ms * 1e-3) / HBM_PEAK}


OVERHEAD_SRC = r'''
extern "C" __global__ void kmap(double* x, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) { double v = x[i]; x[i] = sqrt(sin(v) * sin(v) + cos(v) * cos(v)); }
}
extern "C" __global__ void kprk(const double* x, double* y, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        long il = i == 0 ? n - 1 : i - 1, ir = i == n - 1 ? 0 : i + 1;
        y[i] = (0.5 * x[il] + x[i]) + 0.5 * x[ir];
    }
}
'''


class NativeHip:
    """The same partition benchmark written straight against the HIP runtime
    (the one torch loaded): one stream per partition, async copies and a
    module launch per partition, then a synchronize of every stream
    (`run`); or the layout hx uses (`run_layered`): all copies in on one
    stream, all copies out on another, each partition's kernel on its own
    stream, ordered by HIP events."""

    def __init__(self, parts):
        import ctypes
        import torch
        libdir = os.path.join(os.path.dirname(torch.__file__), "lib")
        self.ct = ctypes
        self.hip = ctypes.CDLL(os.path.join(libdir, "libamdhip64.so"))
        self.streams = []
        for _ in range(parts + 2):
            s = ctypes.c_void_p()
            assert self.hip.hipStreamCreateWithFlags(ctypes.byref(s), 1) == 0
            self.streams.append(s)
        self.h2d, self.d2h = self.streams[parts], self.streams[parts + 1]
        self.streams = self.streams[:parts]
        self.evs = []
        for _ in range(2 * parts):
            e = ctypes.c_void_p()
            assert self.hip.hipEventCreateWithFlags(ctypes.byref(e), 2) == 0  # no timing
            self.evs.append(e)
        self.hip.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self.hip.hipStreamWaitEvent.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint]
        self.hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_int, ctypes.c_void_p]
        self.hip.hipModuleLaunchKernel.argtypes = [ctypes.c_void_p] + [ctypes.c_uint] * 7 + [
            ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p), ctypes.c_void_p]
        self.hip.hipStreamSynchronize.argtypes = [ctypes.c_void_p]
        self.hip.hipStreamDestroy.argtypes = [ctypes.c_void_p]

    def run(self, fn, host_in, host_out, dptrs, bounds):
        ct = self.ct
        keep = []
        for (o, s), d, st in zip(bounds, dptrs, self.streams):
            assert self.hip.hipMemcpyAsync(d, host_in + o * 8, s * 8, 1, st) == 0
            a0, a1 = ct.c_void_p(d), ct.c_int64(s)
            params = (ct.c_void_p * 2)(ct.cast(ct.byref(a0), ct.c_void_p),
                                       ct.cast(ct.byref(a1), ct.c_void_p))
            keep.append((a0, a1, params))
            assert self.hip.hipModuleLaunchKernel(fn, (s + 255) // 256, 1, 1, 256, 1, 1, 0, st,
                                                  params, None) == 0
            assert self.hip.hipMemcpyAsync(host_out + o * 8, d, s * 8, 2, st) == 0
        for st in self.streams:
            assert self.hip.hipStreamSynchronize(st) == 0

    def run_layered(self, fn, host_in, host_out, dptrs, bounds):
        ct, hip = self.ct, self.hip
        keep = []
        for p, ((o, s), d, st) in enumerate(zip(bounds, dptrs, self.streams)):
            e_in, e_k = self.evs[2 * p], self.evs[2 * p + 1]
            assert hip.hipMemcpyAsync(d, host_in + o * 8, s * 8, 1, self.h2d) == 0
            assert hip.hipEventRecord(e_in, self.h2d) == 0
            assert hip.hipStreamWaitEvent(st, e_in, 0) == 0
            a0, a1 = ct.c_void_p(d), ct.c_int64(s)
            params = (ct.c_void_p * 2)(ct.cast(ct.byref(a0), ct.c_void_p),
                                       ct.cast(ct.byref(a1), ct.c_void_p))
            keep.append((a0, a1, params))
            assert hip.hipModuleLaunchKernel(fn, (s + 255) // 256, 1, 1, 256, 1, 1, 0, st,
                                             params, None) == 0
            assert hip.hipEventRecord(e_k, st) == 0
            assert hip.hipStreamWaitEvent(self.d2h, e_k, 0) == 0
            assert hip.hipMemcpyAsync(host_out + o * 8, d, s * 8, 2, self.d2h) == 0
        assert hip.hipStreamSynchronize(self.d2h) == 0

    def close(self):
        for st in self.streams + [self.h2d, self.d2h]:
            self.hip.hipStreamDestroy(st)
        for e in self.evs:
            self.hip.hipEventDestroy(e)


def overhead_in_child():
    """The paper's two overhead experiments, each in a process of its own, as
    the paper ran them as separate programs.  Run after E2 in one context, the
    dependent copy-kernel-copy chain of E1 measured 0.975 ms at 2^21 doubles
    once E2 had run its partitions of 2^24 doubles and more, against 0.65 ms
    before (and 0.62 ms for the raw-stream chain either way); the cause is not
    known."""
    import subprocess
    res = {}
    for which in ("e2", "e1"):
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--overhead-only", which],
                           capture_output=True, text=True, timeout=600)
        sys.stderr.write(r.stderr)
        if r.returncode != 0:
            raise RuntimeError(f"overhead experiment {which} failed ({r.returncode})")
        part = json.loads(r.stdout.strip().splitlines()[-1])
        if which == "e2":
            res.update(part)
        else:
            res["e1_sequential_stencil"] = part["e1_sequential_stencil"]
    res["processes"] = "E2 and E1 each in a child process of their own"
    return res


def overhead_leg(hx, which="e2", parts=4, iters=11):
    """The paper's overhead experiments.  E2 (Sec. V-A.2, Algorithm 1): a vector of
    n = 2^m * 1024 * 256 * 4 doubles (m = 1..8) in `parts` partitions, each
    copied in, mapped by k(x) = sqrt(sin^2 x + cos^2 x) (compiled at run time)
    and copied out, all partitions in flight; the hx future graph against the
    same work on raw HIP streams.  E1 (Sec. V-A.1): the 3-point stencil on one
    vector of 2^21..2^26 doubles as a dependent copy-in, kernel, copy-out
    chain, against the same chain on one raw HIP stream.  Each time is the mean
    of iterations 2..11, the paper's method.  `which` selects the experiment."""
    import torch
    ctx = hx.hx_ctx_create(0)
    prog = hx.hx_program_create(ctx, OVERHEAD_SRC, "partition_kernel.hip")
    hx.hx_program_build(ctx, prog)
    fn = hx.hx_program_function(ctx, prog, "kmap")
    nmax = (1 << 8) * 1024 * 256 * 4
    hin = hx.hx_host_alloc(ctx, nmax * 8)
    hout = hx.hx_host_alloc(ctx, nmax * 8)
    arr = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_double * nmax).from_address(hin))
    arr[:] = np.arange(nmax, dtype=np.float64)
    native = NativeHip(parts)
    rows = []
    for k, m in enumerate([1] + list(range(1, 9)) if which == "e2" else []):  # 1st: warm-up
        n = (1 << m) * 1024 * 256 * 4
        bounds = [(p * n // parts, (p + 1) * n // parts - p * n // parts) for p in range(parts)]
        bufs = [hx.hx_buffer_create(ctx, s * 8) for _, s in bounds]
        dptrs = [hx.hx_buffer_ptr(ctx, b)[0] for b in bufs]

        def run_hx():
            evs, keep = [], []
            for (o, s), b in zip(bounds, bufs):
                e1 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, hin + o * 8, b, 0, 0, 0,
                                                           s * 8))
                e2 = hx.hx_program_run(ctx, prog, "kmap",
                                       [hx.karg_buffer(b), hx.karg_value(np.int64(s))],
                                       ((s + 255) // 256,), (256,), deps=[e1])
                e3 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, hout + o * 8, b, 0, 0, 0,
                                                           s * 8), [e2])
                evs.append(e3)
                keep += [e1, e2]
            w = hx.hx_when_all(ctx, evs)
            assert hx.hx_wait(ctx, w) == hx.HX_OK, hx.hx_last_error(ctx)
            for e in keep + evs + [w]:
                hx.hx_event_release(ctx, e)

        def run_native():
            native.run(fn, hin, hout, dptrs, bounds)

        def run_native_layered():
            native.run_layered(fn, hin, hout, dptrs, bounds)

        res = {}
        for name, f in (("hx", run_hx), ("native", run_native),
                        ("native_layered", run_native_layered)):
            ts = []
            for _ in range(iters):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f()
                ts.append(time.perf_counter() - t0)
            res[name] = float(np.mean(ts[1:])) * 1e3
        out = np.ctypeslib.as_array((np.ctypeslib.ctypes.c_double * n).from_address(hout))
        err = float(np.max(np.abs(out[:: max(1, n // 4096)] - 1.0)))
        for b in bufs:
            hx.hx_buffer_destroy(ctx, b)
        if k == 0:
            continue
        rows.append({"m": m, "n": n, "hx_ms": res["hx"], "native_ms": res["native"],
                     "hx_over_native": res["hx"] / res["native"],
                     "native_layered_ms": res["native_layered"],
                     "hx_over_native_layered": res["hx"] / res["native_layered"],
                     "host_link_GBps_hx": 2 * n * 8 / (res["hx"] * 1e-3) / 1e9,
                     "max_abs_err_vs_1": err})
        log(f"overhead m={m} n={n}: hx {res['hx']:.3f} ms, native {res['native']:.3f} ms, "
            f"native with hx's stream layout {res['native_layered']:.3f} ms")
    # E1 (Sec. V-A.1): the 3-point stencil, one vector, copy in -> kernel ->
    # copy out as a dependent chain, against the same chain with synchronous
    # HIP calls.
    kprk = hx.hx_program_function(ctx, prog, "kprk")
    e1_rows = []
    for k, m in enumerate([1] + list(range(1, 7)) if which == "e1" else []):
        n = (1 << m) * 1024 * 256 * 4
        bx = hx.hx_buffer_create(ctx, n * 8)
        by = hx.hx_buffer_create(ctx, n * 8)
        px, py = hx.hx_buffer_ptr(ctx, bx)[0], hx.hx_buffer_ptr(ctx, by)[0]

        def submit_chain():
            e1 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_H2D, hin, bx, 0, 0, 0, n * 8))
            e2 = hx.hx_program_run(ctx, prog, "kprk",
                                   [hx.karg_buffer(bx, 0, hx.HX_ACCESS_READ),
                                    hx.karg_buffer(by, 0, hx.HX_ACCESS_WRITE),
                                    hx.karg_value(np.int64(n))], ((n + 255) // 256,), (256,),
                                   deps=[e1])
            e3 = hx.hx_copy_async(ctx, hx.hx_copy_desc(hx.HX_D2H, hout, by, 0, 0, 0, n * 8), [e2])
            return (e1, e2, e3)

        def run_hx():
            evs = submit_chain()
            assert hx.hx_wait(ctx, evs[-1]) == hx.HX_OK
            for e in evs:
                hx.hx_event_release(ctx, e)

        # the same chain captured once as a graph, replayed
        hx.hx_graph_begin(ctx)
        for e in submit_chain():
            hx.hx_event_release(ctx, e)
        graph = hx.hx_graph_end(ctx)

        def run_graph():
            e = hx.hx_graph_launch(ctx, graph)
            assert hx.hx_wait(ctx, e) == hx.HX_OK
            hx.hx_event_release(ctx, e)

        def run_native():
            ct = native.ct
            st = native.streams[0]
            assert native.hip.hipMemcpyAsync(px, hin, n * 8, 1, st) == 0
            a0, a1, a2 = ct.c_void_p(px), ct.c_void_p(py), ct.c_int64(n)
            params = (ct.c_void_p * 3)(*[ct.cast(ct.byref(v), ct.c_void_p) for v in (a0, a1, a2)])
            assert native.hip.hipModuleLaunchKernel(kprk, (n + 255) // 256, 1, 1, 256, 1, 1, 0, st,
                                                    params, None) == 0
            assert native.hip.hipMemcpyAsync(hout, py, n * 8, 2, st) == 0
            assert native.hip.hipStreamSynchronize(st) == 0

        res = {}
        for name, f in (("hx", run_hx), ("native", run_native), ("hx_graph", run_graph)):
            ts = []
            for _ in range(iters):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                f()
                ts.append(time.perf_counter() - t0)
            res[name] = float(np.mean(ts[1:])) * 1e3
        hx.hx_plan_destroy(ctx, graph)
        for b in (bx, by):
            hx.hx_buffer_destroy(ctx, b)
        if k == 0:
            continue
        e1_rows.append({"m": m, "n": n, "hx_ms": res["hx"], "native_ms": res["native"],
                        "hx_over_native": res["hx"] / res["native"],
                        "hx_graph_ms": res["hx_graph"],
                        "hx_graph_over_native": res["hx_graph"] / res["native"]})
        log(f"overhead E1 m={m} n={n}: hx {res['hx']:.3f} ms, native {res['native']:.3f} ms, "
            f"hx graph replay {res['hx_graph']:.3f} ms")
    native.close()
    hx.hx_program_destroy(ctx, prog)
    hx.hx_host_free(ctx, hin)
    hx.hx_host_free(ctx, hout)
    hx.hx_ctx_destroy(ctx)
    return {"parts": parts, "dtype": "f64", "iterations": iters, "rows": rows,
            "e1_sequential_stencil": e1_rows}


def host_cpu():
    """The host's processor model and the CPU counts this process sees."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu_model": model, "nproc": avail, "logical_cpus": os.cpu_count()}


def cpu_baseline(value, seconds, n, T):
    """The oracle, untuned, on one host core over the whole headline workload
    (timed in main while it checks every cell of one GPU pass)."""
    return {"value": value, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"the whole workload: periodic vector of {n} cells (the 64 partitions "
                      f"joined), {T} steps, serial FP64 C oracle, {seconds:.2f} s",
            **host_cpu()}


def oracle_timings():
    """The serial FP64 oracle on one core over a bounded sample of each of the
    other workloads (the per-cell work does not depend on the sample's size),
    in cell-updates/s."""
    import oracle
    import workloads
    res = {}

    def timed(fn):
        t0 = time.perf_counter()
        fn()
        return time.perf_counter() - t0

    s1 = workloads.Periodic1D()
    u = workloads.periodic1d_u0(s1).astype(np.float64)
    t = timed(lambda: oracle.heat1d_periodic(u, s1.r, s1.steps))
    res["periodic_fp64"] = {"value": s1.n * s1.steps / t, "seconds": t,
                            "sample": f"the whole workload: 2^20 cells, {s1.steps} steps"}
    s3 = workloads.Batched1D()
    sizes, rs, _ = workloads.batched1d_problems(s3)
    k = int(np.searchsorted(np.cumsum(sizes), 1 << 26)) + 1
    u = workloads.batched1d_u0(s3, total=int(sizes[:k].sum())).astype(np.float64)
    t = timed(lambda: oracle.heat1d_batched(sizes[:k], rs[:k], u, s3.steps))
    res["batched"] = {"value": float(sizes[:k].sum()) * s3.steps / t, "seconds": t,
                      "sample": f"the first {k} of {s3.count} problems "
                                f"({int(sizes[:k].sum())} cells), {s3.steps} steps"}
    s4 = workloads.Banded2D()
    rows = 1024
    u = workloads.gaussian_bumps(rows, s4.nx, 4, s4.sigma, 4, np.float64)
    st4 = 16
    t = timed(lambda: oracle.heat2d_dirichlet(u, s4.r, st4))
    res["banded_2d"] = {"value": rows * s4.nx * st4 / t, "seconds": t,
                        "sample": f"one band of {rows} x {s4.nx} cells, {st4} steps"}
    s5 = workloads.VarCoef2D()
    m = 1024
    z = workloads.rng(5, 0).standard_normal((m, m))
    kap = np.minimum(np.exp(s5.mu + s5.sigma_log * z), s5.kappa_max)
    u0 = workloads.gaussian_bumps(m, m, 4, s5.sigma, 5, np.float64)
    y = workloads.rng(5, 1).random((m, m))
    t = timed(lambda: oracle.heatvc_grad(u0, kap, y, s5.dt, s5.steps, s5.ckpt))
    res["adjoint"] = {"value": m * m * s5.steps / t, "seconds": t,
                      "unit_note": "forward steps per second of the whole gradient (forward, "
                                   "checkpointed recompute and adjoint sweep)",
                      "sample": f"{m} x {m} cells, {s5.steps} steps, checkpoints every "
                                f"{s5.ckpt}"}
    res["cores"] = 1
    res["unit"] = "cell-updates/s"
    log(f"oracle timings: {res}")
    return res


if __name__ == "__main__":
    main()
