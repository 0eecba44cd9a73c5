"""The coupled loop of Alg. coupled_EL on one GPU: each step the particles
advance between the two retained velocity levels while the field producer
computes the next level, which then replaces the older one.

Scheduling only (no arithmetic of the method).  With ``streams=1`` (the
default) the field producer (libns2d.so) and the particle library
(liblpt.so) share the null stream and the sequence runs in stream order.
With ``streams=2`` they run on two HIP streams so that the field step and
the particle step may overlap; two events keep the hand-off in order: the
particle stream waits for the new level before ingesting it, and the field
stream waits for that ingest before its next step overwrites the velocity
buffers.  Measured at 2048^2 with 2^20 FP64 tracers, the overlap is slower
(329 against 298 us a coupled step): both phases contend for HBM and L2.
"""
from __future__ import annotations

from . import lpt, ns2d


class CoupledLoop:
    def __init__(self, n, nu, dt, omega0, precision="fp64", length=0.0, streams=1,
                 transforms="auto", **tracker_kw):
        import torch
        assert streams in (1, 2)
        self.dt = dt
        self.steps = 0
        if streams == 2:
            self._sp, self._sf = torch.cuda.Stream(), torch.cuda.Stream()
            hp, hf = self._sp.cuda_stream, self._sf.cuda_stream
        else:
            self._sp = self._sf = None
            hp = hf = None
        self.field = ns2d.Ns2d(n, nu, dt, length=length, stream=hf, transforms=transforms)
        self.tracker = lpt.Tracker(n, precision, length=length, stream=hp, **tracker_kw)
        self.tracker.set_time_mode("pingpong")
        self.field.set_vorticity(omega0)
        self.field.synchronize()
        self.tracker.set_snapshot_device(0, 0.0, *self.field.velocity_ptrs())
        self.tracker.synchronize()
        self.field.step(1)
        self.field.synchronize()
        self.tracker.set_snapshot_device(1, dt, *self.field.velocity_ptrs())
        self.tracker.synchronize()
        self._ev_level = torch.cuda.Event()
        self._ev_taken = torch.cuda.Event()

    def step(self, count=1, stats_every=0):
        """`count` coupled steps: particle step s between levels s and s+1,
        field step to level s+2, level s+2 into the slot of level s."""
        for _ in range(count):
            s = self.steps
            self.tracker.step(1, self.dt, stats_every)
            self.field.step(1)
            if self._sp is not None:
                self._ev_level.record(self._sf)
                self._sp.wait_event(self._ev_level)
            self.tracker.set_snapshot_device(s % 2, (s + 2) * self.dt, *self.field.velocity_ptrs())
            if self._sp is not None:
                self._ev_taken.record(self._sp)
                self._sf.wait_event(self._ev_taken)
            self.steps += 1

    def record_event(self, event):
        """Record `event` where all work enqueued so far has finished (the
        particle stream waits on every field step)."""
        if self._sp is not None:
            event.record(self._sp)
        else:
            event.record()

    def synchronize(self):
        self.tracker.synchronize()
        self.field.synchronize()

    def close(self):
        self.synchronize()
        self.tracker.close()
        self.field.close()
