"""Host-to-host run of a 2D row-band grid over many passes, composed from the
library's futures: argument marshalling and graph construction only; every
copy and kernel runs in the library.

The partition benchmark of Sec. V-A.2 (Algorithm 1) copies each partition in,
runs a kernel on it and copies it out, with all partitions in flight.  For a
run of T steps that needs several kernel passes, the literal per-pass graph
(band p's pass b waits for bands p-1..p+1 at pass b-1) makes a band's last
pass depend on every band within T rows, that is on the whole grid's input,
so no copy out could start before every copy in.  Pipeline2D instead gives
each band an extended input of its own rows plus T halo rows on each side
(the band's light cone over T steps):

  H2D(p)       host rows of band p -> the middle of ext[p]
  halo(p, -1)  D2D: the last T own rows of ext[p-1] -> the top T rows of ext[p]
  halo(p, +1)  D2D: the first T own rows of ext[p+1] -> the bottom T rows
  K(p)         hx_launch_stencil over ext[p] (T steps, passes of time_block,
               zero-Dirichlet at the extended edges), into out[p]
  D2H(p)       the own rows of out[p] -> host rows of band p

K(p) depends only on H2D(p-1), H2D(p) and the first T rows of H2D(p+1)
(through the halo copies), and D2H(p) on K(p): copies out of early bands run
while later bands are still copied in.  Each band after the first is copied
in as two copies, its first T rows (the halo its upper neighbour reads) and
then the rest, so K(p) need not wait for all of band p+1 to arrive: the first
copy out, which every later one queues behind, starts a band's copy time
earlier.  The extended edges' wrong boundary values move inward one row per
step, so after T steps they have reached exactly the T halo rows and the own
rows equal the whole-grid run (the grid's true top and bottom edges have no
halo: there the zero-Dirichlet edge is the real one).  The cost is the
recomputation of 2T halo rows per band.  A kernel launch never writes its
input, so the halo copies out of ext[p] need no ordering against K(p).
"""
from __future__ import annotations

from . import (HX_BC_DIRICHLET0, HX_D2D, HX_D2H, HX_F32, HX_H2D, hx_buffer_create,
               hx_buffer_destroy, hx_copy_async, hx_copy_desc, hx_event_release,
               hx_launch_stencil, hx_when_all, stencil_args)


class Pipeline2D:
    """A zero-Dirichlet ny x nx f32 grid (row-major) in `bands` row bands
    (`bounds`: (first row, rows) per band), advanced `steps` steps at rate r.
    Device buffers are allocated once here (three extended bands each)."""

    def __init__(self, ctx, ny, nx, bounds, steps, r, time_block=16, cells_per_lane=4,
                 rows_per_block=128):
        self.ctx, self.ny, self.nx, self.bounds = ctx, ny, nx, list(bounds)
        self.steps, self.r = steps, r
        self.tb, self.cpl, self.rows = time_block, cells_per_lane, rows_per_block
        P = len(self.bounds)
        self.top = [min(steps, o) for o, _ in self.bounds]             # halo rows above
        self.bot = [min(steps, ny - (o + s)) for o, s in self.bounds]  # halo rows below
        self.ext_rows = [t + s + b for t, (_, s), b in zip(self.top, self.bounds, self.bot)]
        rb = nx * 4
        self.ext = [hx_buffer_create(ctx, e * rb) for e in self.ext_rows]
        self.out = [hx_buffer_create(ctx, e * rb) for e in self.ext_rows]
        self.tmp = [hx_buffer_create(ctx, e * rb) for e in self.ext_rows]
        for p in range(P - 1):  # halos come from the adjacent band only
            if self.bounds[p + 1][1] < self.bot[p] or self.bounds[p][1] < self.top[p + 1]:
                self.close()
                raise ValueError("every band needs at least `steps` rows")

    def run(self, host_in: int, host_out: int, kernels=True, deps=()):
        """Queue the whole run from host_in to host_out (ny x nx f32 each,
        pinned for overlap, caller-owned until the final event completes);
        `deps` gate the copies in (a run reuses the device buffers, so a
        second run must follow the first's final event).  Returns (final
        event, H2D events, kernel events, D2H events): the H2D events in
        submission order, one or two per band (self.h2d_index[p] lists band
        p's, the last of which completes after the others), one kernel and one
        D2H event per band (no kernel events when kernels is False: then each
        band's input rows go straight back out, the copies alone).  The caller
        releases the events."""
        ctx, rb = self.ctx, self.nx * 4
        P = len(self.bounds)
        h2d, ker, d2h = [], [], []
        head, whole = [], []  # per band: the copy of its first rows, and of all of it
        self.h2d_index = []

        def queue_band(p):
            o, s = self.bounds[p]
            halos = []
            if kernels and self.top[p]:
                q = p - 1
                src = (self.top[q] + self.bounds[q][1] - self.top[p]) * rb
                halos.append(hx_copy_async(ctx, hx_copy_desc(HX_D2D, 0, self.ext[p], 0,
                                                             self.ext[q], src, self.top[p] * rb),
                                           [whole[q]]))
            if kernels and self.bot[p]:
                # chained on the top halo's copy: the runtime continues the
                # compute stream whose last operation is a dependency, so a
                # band's halo copies and kernel share one stream and the next
                # band starts on the other, instead of a halo copy queueing
                # behind the previous band's kernel
                q = p + 1
                dst = (self.top[p] + s) * rb
                halos.append(hx_copy_async(ctx, hx_copy_desc(HX_D2D, 0, self.ext[p], dst,
                                                             self.ext[q], self.top[q] * rb,
                                                             self.bot[p] * rb),
                                           [head[q]] + halos[-1:]))
            if kernels:
                k = hx_launch_stencil(ctx, self._kernel_args(p), [whole[p]] + halos)
                ker.append(k)
                src_buf, dep = self.out[p], k
            else:
                src_buf, dep = self.ext[p], whole[p]
            for e in halos:
                hx_event_release(ctx, e)
            d2h.append(hx_copy_async(ctx, hx_copy_desc(HX_D2H, host_out + o * rb, src_buf,
                                                       self.top[p] * rb, 0, 0, s * rb),
                                     [dep]))

        # copies in, in band order; band p is queued as soon as band p+1's
        # copy in (its last dependency) has been
        for p in range(P):
            o, s = self.bounds[p]
            first = self.bot[p - 1] if kernels and p >= 1 and self.bot[p - 1] < s else 0
            idx = []
            if first:
                # the rows band p-1 reads as its bottom halo, then the rest
                # (ordered after them, so its event stands for the whole band)
                e = hx_copy_async(ctx, hx_copy_desc(HX_H2D, host_in + o * rb, self.ext[p],
                                                    self.top[p] * rb, 0, 0, first * rb),
                                  list(deps))
                idx.append(len(h2d))
                h2d.append(e)
                head.append(e)
                e = hx_copy_async(ctx, hx_copy_desc(HX_H2D, host_in + (o + first) * rb,
                                                    self.ext[p], (self.top[p] + first) * rb,
                                                    0, 0, (s - first) * rb),
                                  list(deps) + [e])
            else:
                e = hx_copy_async(ctx, hx_copy_desc(HX_H2D, host_in + o * rb, self.ext[p],
                                                    self.top[p] * rb, 0, 0, s * rb),
                                  list(deps))
                head.append(e)
            idx.append(len(h2d))
            h2d.append(e)
            whole.append(e)
            self.h2d_index.append(idx)
            if p >= 1:
                queue_band(p - 1)
        queue_band(P - 1)
        final = hx_when_all(ctx, d2h)
        return final, h2d, ker, d2h

    def _kernel_args(self, p):
        return stencil_args(dims=2, dtype=HX_F32, nx=self.nx, ny=self.ext_rows[p],
                            steps=self.steps, r=self.r, inp=self.ext[p], out=self.out[p],
                            tmp=self.tmp[p], bc_lo=HX_BC_DIRICHLET0, bc_hi=HX_BC_DIRICHLET0,
                            time_block=self.tb, cells_per_lane=self.cpl,
                            rows_per_block=self.rows)

    def kernels_only(self, deps=()):
        """The kernels alone, on the extended inputs a previous run left in
        place; returns (final event, kernel events)."""
        ker = [hx_launch_stencil(self.ctx, self._kernel_args(p), list(deps))
               for p in range(len(self.bounds))]
        return hx_when_all(self.ctx, ker), ker

    def close(self):
        for b in self.ext + self.out + self.tmp:
            hx_buffer_destroy(self.ctx, b)
        self.ext, self.out, self.tmp = [], [], []
