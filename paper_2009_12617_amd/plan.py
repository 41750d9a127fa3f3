"""Python binding of the SPME step: torch tensors in, the C ABI underneath.

PyTorch supplies device memory and the stream; every step of the SPME path
runs in libspme.so's HIP kernels.  There is no CPU fallback: without the
built library or a GPU, construction raises.
"""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (PME_EBUSY, PME_FP32_FIXED, PME_FP32_FIXED_BF16, PME_FP32_FIXED_HALF, PME_FP64,
                   SystemDesc, Tuning, check)

KERNEL_NAMES = ("bin", "spread_x", "convolve_yz", "interpolate")
# pme_step_probe: which kernel a probe step launches twice
PROBE = {"none": 0, "bin": 1, "spread_x": 2, "convolve_yz": 3, "interpolate": 4, "clear": 5}
PRECISIONS = {"fp32_fixed": PME_FP32_FIXED, "fp64": PME_FP64,
              "fp32_fixed_half": PME_FP32_FIXED_HALF, "fp32_fixed_bf16": PME_FP32_FIXED_BF16}


def _box9(box):
    b = np.asarray(box, dtype=np.float64)
    if b.shape == (3,):
        b = np.diag(b)
    b = np.ascontiguousarray(b.reshape(9))
    return (ctypes.c_double * 9)(*b.tolist())


def _dev_f64(t, shape, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def grid3(K):
    """(K1, K2, K3) from a cubic K or a 3-sequence of grid points along x, y, z."""
    if np.ndim(K) == 0:
        return (int(K),) * 3
    k = tuple(int(v) for v in K)
    if len(k) != 3:
        raise ValueError("K must be an int or three grid sizes (K1, K2, K3)")
    return k


class Plan:
    """One SPME reciprocal-space solver on a K1 x K2 x K3 grid (K: an int for
    a cubic grid, or (K1, K2, K3) along x, y, z).

    precision: "fp32_fixed" (FP32 splines/FFT/convolution, 64-bit fixed-point
    charge grid, FP64 moduli/energy/virial), "fp32_fixed_half" (the same with
    the half spectrum stored in binary16 between launches), "fp32_fixed_bf16"
    (the same in bfloat16) or "fp64".
    """

    def __init__(self, K, order=4, beta=0.34, max_atoms=0, precision="fp32_fixed",
                 frac_bits=32, coulomb=1.0, device=None, stream=None):
        lib = _lib.load()
        if precision not in PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(PRECISIONS)}")
        self.grid = grid3(K)  # (K1, K2, K3)
        self.order, self.beta = int(order), float(beta)
        self.max_atoms, self.precision = int(max_atoms), precision
        self.frac_bits = int(frac_bits)
        self.coulomb = float(coulomb)
        prec = PRECISIONS[precision]
        self.device = torch.device(device if device is not None else "cuda")
        if self.device.type != "cuda":
            raise ValueError("the SPME step runs on a GPU device")
        nbytes = lib.pme_workspace_bytes(*self.grid, self.order, self.max_atoms, prec)
        if nbytes == 0:
            raise _lib.SpmeError(2, f"pme_workspace_bytes(K={K}, order={order})")
        self.workspace_bytes = nbytes
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = (self._ws.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(lib.pme_create(ctypes.byref(h), *self.grid, self.order, self.beta,
                             self.max_atoms, prec, self.frac_bits, self.coulomb, base, nbytes,
                             ctypes.c_void_p(self.stream.cuda_stream)), "pme_create")
        self._h = h
        self._lib = lib
        self._keep = ()
        self._n = 0

    @staticmethod
    def workspace_bytes_for(K, order, max_atoms, precision="fp32_fixed"):
        """Device workspace a plan with these parameters needs (0 if unsupported)."""
        lib = _lib.load()
        return int(lib.pme_workspace_bytes(*grid3(K), int(order), int(max_atoms),
                                           PRECISIONS[precision]))

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pme_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        self.stream = stream
        check(self._lib.pme_set_stream(self._h, ctypes.c_void_p(stream.cuda_stream)), "pme_set_stream")

    # -- the step -----------------------------------------------------------
    def spread(self, pos, q, box):
        n = int(q.shape[0])
        _dev_f64(pos, (n, 3), "pos")
        _dev_f64(q, (n,), "q")
        self._keep = (pos, q)
        self._n = n
        check(self._lib.pme_spread(self._h, pos.data_ptr(), q.data_ptr(), n, _box9(box)),
              "pme_spread")

    def solve(self, ev=None):
        if ev is None:
            ev = torch.empty(7, dtype=torch.float64, device=self.device)
        _dev_f64(ev, (7,), "ev")
        check(self._lib.pme_solve(self._h, ev.data_ptr()), "pme_solve")
        return ev

    def gather(self, forces=None, accumulate=False):
        if forces is None:
            forces = torch.empty((self._n, 3), dtype=torch.float64, device=self.device)
        _dev_f64(forces, (self._n, 3), "forces")
        check(self._lib.pme_gather(self._h, forces.data_ptr(), int(bool(accumulate))),
              "pme_gather")
        return forces

    def step(self, pos, q, box, forces=None, accumulate=False, ev=None):
        """Forces [N,3] and ev = [E, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz] (device float64)."""
        n = int(q.shape[0])
        _dev_f64(pos, (n, 3), "pos")
        _dev_f64(q, (n,), "q")
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if ev is None:
            ev = torch.empty(7, dtype=torch.float64, device=self.device)
        _dev_f64(forces, (n, 3), "forces")
        _dev_f64(ev, (7,), "ev")
        self._keep = (pos, q)
        self._n = n
        check(self._lib.pme_step(self._h, pos.data_ptr(), q.data_ptr(), n, _box9(box),
                                 forces.data_ptr(), int(bool(accumulate)), ev.data_ptr()),
              "pme_step")
        return forces, ev

    def step_probe(self, pos, q, box, forces, ev, repeat):
        """pme_step_probe: a step with one kernel launched twice (timing
        diagnostics; repeat is one of PROBE)."""
        n = int(q.shape[0])
        _dev_f64(pos, (n, 3), "pos")
        _dev_f64(q, (n,), "q")
        _dev_f64(forces, (n, 3), "forces")
        _dev_f64(ev, (7,), "ev")
        self._keep = (pos, q)
        self._n = n
        check(self._lib.pme_step_probe(self._h, pos.data_ptr(), q.data_ptr(), n, _box9(box),
                                       forces.data_ptr(), ev.data_ptr(), int(repeat)),
              "pme_step_probe")

    def bind(self, pos, q, box, forces=None, ev=None, accumulate=False):
        """Bind the buffers of this plan's batched steps (see Batch); returns (forces, ev)."""
        n = int(q.shape[0])
        _dev_f64(pos, (n, 3), "pos")
        _dev_f64(q, (n,), "q")
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if ev is None:
            ev = torch.empty(7, dtype=torch.float64, device=self.device)
        _dev_f64(forces, (n, 3), "forces")
        _dev_f64(ev, (7,), "ev")
        check(self._lib.pme_bind(self._h, pos.data_ptr(), q.data_ptr(), n, _box9(box),
                                 forces.data_ptr(), int(bool(accumulate)), ev.data_ptr()),
              "pme_bind")
        self._bound = (pos, q, forces, ev)
        self._n = n
        return forces, ev

    # -- kernel variants ------------------------------------------------------
    @property
    def tuning(self):
        """The plan's kernel variants: {"conv", "interp", "bin_chunk"}."""
        t = Tuning()
        check(self._lib.pme_get_tuning(self._h, ctypes.byref(t)), "pme_get_tuning")
        return t.as_dict()

    def set_tuning(self, conv=None, interp=None, bin_chunk=None):
        cur = self.tuning
        t = Tuning(cur["conv"] if conv is None else int(conv),
                   cur["interp"] if interp is None else int(interp),
                   cur["bin_chunk"] if bin_chunk is None else int(bin_chunk))
        check(self._lib.pme_set_tuning(self._h, ctypes.byref(t)), "pme_set_tuning")

    def variants(self):
        """PME_VAR_* bits of the variants this plan's shape can run."""
        prec = PRECISIONS[self.precision]
        return int(self._lib.pme_tuning_variants(*self.grid, self.order, prec))

    def autotune(self, pos, q, box, reps=20, forces=None, ev=None):
        """Measure every supported variant on these inputs (pme_autotune) and
        keep the fastest.  Returns {"best": tuning, "us": best us/step,
        "candidates": [(tuning, us or None), ...]}."""
        n = int(q.shape[0])
        _dev_f64(pos, (n, 3), "pos")
        _dev_f64(q, (n,), "q")
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        if ev is None:
            ev = torch.empty(7, dtype=torch.float64, device=self.device)
        _dev_f64(forces, (n, 3), "forces")
        _dev_f64(ev, (7,), "ev")
        best = Tuning()
        best_us = ctypes.c_double(0.0)
        times = (ctypes.c_double * len(TUNE_CANDIDATES))()
        self._keep = (pos, q)
        self._n = n
        check(self._lib.pme_autotune(self._h, pos.data_ptr(), q.data_ptr(), n, _box9(box),
                                     forces.data_ptr(), ev.data_ptr(), int(reps), ctypes.byref(best),
                                     ctypes.byref(best_us), times, len(TUNE_CANDIDATES)),
              "pme_autotune")
        cands = [(dict(c), (None if times[i] < 0 else float(times[i])))
                 for i, c in enumerate(TUNE_CANDIDATES)]
        return {"best": best.as_dict(), "us": float(best_us.value), "candidates": cands}

    # -- inspection -----------------------------------------------------------
    def set_debug(self, keep_charge_grid=True):
        check(self._lib.pme_set_debug(self._h, int(bool(keep_charge_grid))), "pme_set_debug")

    def debug_grid(self, which):
        """0: charge grid (int64 fixed point or float64) [z, y, x], 1: half
        spectrum (complex) as columns [x', z, y] of shape [K1/2+1, K3, K2]
        (bfloat16 plans: real and imaginary parts as a trailing axis of 2),
        2: potential phi [z, y, x]."""
        K1, K2, K3 = self.grid
        kh = K1 // 2 + 1
        fx = self.precision != "fp64"
        if which == 0:
            out = torch.empty((K3, K2, K1), dtype=torch.int64 if fx else torch.float64,
                              device=self.device)
        elif which == 1:
            if self.precision == "fp32_fixed_bf16":  # torch has no bfloat16 complex type
                out = torch.empty((kh, K3, K2, 2), dtype=torch.bfloat16, device=self.device)
            else:
                dt = {"fp32_fixed": torch.complex64, "fp32_fixed_half": torch.complex32,
                      "fp64": torch.complex128}[self.precision]
                out = torch.empty((kh, K3, K2), dtype=dt, device=self.device)
        elif which == 2:
            out = torch.empty((K3, K2, K1), dtype=torch.float32 if fx else torch.float64,
                              device=self.device)
        else:
            raise ValueError("which must be 0, 1 or 2")
        assert out.numel() * out.element_size() == self._lib.pme_debug_grid_bytes(self._h, which)
        check(self._lib.pme_debug_grid(self._h, int(which), out.data_ptr()), "pme_debug_grid")
        return out

    def check(self):
        """Synchronise; return the sticky flags and clear them (raises on none)."""
        flags = ctypes.c_uint(0)
        rc = self._lib.pme_check(self._h, ctypes.byref(flags))
        if rc not in (0, 4, 6, 7):
            check(rc, "pme_check")
        return int(flags.value)

    def kernel_timing(self, enable=True):
        """Events attached to every dispatch (host-launched steps)."""
        check(self._lib.pme_kernel_timing(self._h, int(bool(enable))), "pme_kernel_timing")

    def kernel_times(self):
        """Accumulated per-kernel milliseconds since the last call, and the step count."""
        ms = (ctypes.c_double * len(KERNEL_NAMES))()
        steps = ctypes.c_int(0)
        check(self._lib.pme_kernel_times(self._h, ms, len(KERNEL_NAMES), ctypes.byref(steps)),
              "pme_kernel_times")
        return dict(zip(KERNEL_NAMES, list(ms))), int(steps.value)


# Candidate order of pme_autotune: conv x interp x bin_chunk, bin_chunk fastest.
TUNE_CANDIDATES = tuple({"conv": c, "interp": i, "bin_chunk": b}
                        for c in (0, 1, 2) for i in (0, 1) for b in (256, 512, 1024))


class Batch:
    """One step of many bound plans per run: plans that share precision, grid
    and spline order share every kernel launch (pme_batch_run)."""

    def __init__(self, plans, stream=None):
        self.plans = list(plans)
        for pl in self.plans:
            if getattr(pl, "_bound", None) is None:
                raise RuntimeError("every plan of a batch must be bound first (Plan.bind)")
        self._lib = _lib.load()
        self._handles = (ctypes.c_void_p * len(self.plans))(*[pl._h.value for pl in self.plans])
        self.stream = stream

    def run(self, stream=None):
        st = stream or self.stream or torch.cuda.current_stream()
        check(self._lib.pme_batch_run(self._handles, len(self.plans), ctypes.c_void_p(st.cuda_stream)),
              "pme_batch_run")


class BatchPool:
    """Resident systems in one device arena (pme_batch_*): admission by
    footprint, a slot per system, one step of any set of slots per launch.

    Each admitted system owns device buffers carved from the arena
    (positions, charges, forces, energy/virial) unless the caller passes its
    own tensors.  All work is enqueued on `stream`."""

    def __init__(self, arena_bytes, max_systems=256, device=None, stream=None):
        self._lib = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        self.arena_bytes = int(arena_bytes)
        self._arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=self.device)
        base = (self._arena.data_ptr() + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        check(self._lib.pme_batch_create(ctypes.byref(h), int(max_systems), base, self.arena_bytes,
                                         ctypes.c_void_p(self.stream.cuda_stream)),
              "pme_batch_create")
        self._h = h
        self._io = {}    # slot -> (pos, q, forces, ev) tensors
        self._n, self._box = {}, {}  # slot -> bound atom count and box
        self._grid, self._order, self._prec = {}, {}, {}
        self._keep = {}  # slot -> caller tensors kept alive

    @staticmethod
    def desc(K, order, beta, max_atoms, precision="fp32_fixed", box=None, n=None):
        d = SystemDesc()
        d.K1, d.K2, d.K3 = grid3(K)
        d.order, d.beta = int(order), float(beta)
        d.precision = PRECISIONS[precision]
        d.max_atoms = int(max_atoms)
        d.N = int(max_atoms if n is None else n)
        b = np.eye(3) if box is None else np.asarray(box, dtype=np.float64)
        if b.shape == (3,):
            b = np.diag(b)
        d.box[:] = [float(v) for v in b.reshape(9)]
        return d

    @staticmethod
    def footprint(K, order, max_atoms, precision="fp32_fixed", own_buffers=True):
        """Arena bytes a system takes (with its buffers carved from the arena
        when own_buffers)."""
        d = BatchPool.desc(K, order, 1.0, max_atoms, precision)
        if not own_buffers:
            d.pos = 1  # any non-NULL pointer: the caller's buffers
        return int(_lib.load().pme_batch_footprint(ctypes.byref(d)))

    def admit(self, K, order, beta, box, max_atoms, n=None, precision="fp32_fixed"):
        """Admit a system with arena-carved buffers; returns the slot, or None
        when no slot or arena range is free (PME_EBUSY)."""
        d = self.desc(K, order, beta, max_atoms, precision, box, n)
        slot = ctypes.c_int(-1)
        rc = self._lib.pme_batch_admit(self._h, ctypes.byref(d), ctypes.byref(slot))
        if rc == PME_EBUSY:
            return None
        check(rc, "pme_batch_admit")
        s = int(slot.value)
        self._io[s] = self._wrap_io(s, int(max_atoms))
        self._n[s] = int(max_atoms if n is None else n)
        self._box[s] = np.asarray(box, dtype=np.float64)
        self._grid[s], self._order[s], self._prec[s] = grid3(K), int(order), PRECISIONS[precision]
        return s

    def _wrap_io(self, slot, max_atoms):
        ptrs = [ctypes.c_void_p() for _ in range(4)]
        check(self._lib.pme_batch_io(self._h, slot, *[ctypes.byref(p) for p in ptrs]), "pme_batch_io")
        views = []
        for p, shape in zip(ptrs, ((max_atoms, 3), (max_atoms,), (max_atoms, 3), (7,))):
            off = p.value - self._arena.data_ptr()  # byte offset into the arena tensor
            nel = int(np.prod(shape))
            views.append(self._arena[off:off + 8 * nel].view(torch.float64).view(*shape))
        return tuple(views)

    def io(self, slot):
        """(pos, q, forces, ev) device tensors of an admitted slot."""
        return self._io[slot]

    def results_span(self, slot):
        """(span, ev_offset): a uint8 device view of the arena from the slot's
        forces to the end of its energy/virial vector, so that one copy
        fetches both, and the byte offset of the energy/virial vector in it;
        None when they are not carved one after the other."""
        _, _, f, ev = self._io[slot]
        base = self._arena.data_ptr()
        of, oe = f.data_ptr() - base, ev.data_ptr() - base
        if oe < of + f.numel() * 8 or oe - of - f.numel() * 8 >= 256:
            return None
        return self._arena[of:oe + 56], oe - of

    def update(self, slot, n, box):
        """New atom count and box of a slot whose buffers live in the arena."""
        check(self._lib.pme_batch_update(self._h, int(slot), None, None, int(n), _box9(box), None, None),
              "pme_batch_update")
        self._n[slot] = int(n)
        self._box[slot] = np.asarray(box, dtype=np.float64)

    def retire(self, slot):
        check(self._lib.pme_batch_retire(self._h, int(slot)), "pme_batch_retire")
        for d in (self._io, self._keep, self._n, self._box, self._grid, self._order, self._prec):
            d.pop(slot, None)

    def launch(self, slots=None):
        """One step of the listed slots (None: every admitted system)."""
        if slots is None:
            check(self._lib.pme_batch_launch(self._h, None, 0), "pme_batch_launch")
            return
        arr = (ctypes.c_int * len(slots))(*[int(s) for s in slots])
        check(self._lib.pme_batch_launch(self._h, arr, len(slots)), "pme_batch_launch")

    def stats(self):
        n = ctypes.c_int(0)
        used = ctypes.c_size_t(0)
        lf = ctypes.c_size_t(0)
        check(self._lib.pme_batch_stats(self._h, ctypes.byref(n), ctypes.byref(used), ctypes.byref(lf)),
              "pme_batch_stats")
        return {"admitted": int(n.value), "bytes_used": int(used.value), "largest_free": int(lf.value)}

    def set_tuning(self, slot, conv=None, interp=None, bin_chunk=None):
        """Kernel variants of an admitted system's plan (pme_set_tuning); a
        batched launch groups systems whose variants agree."""
        h = self._lib.pme_batch_plan(self._h, int(slot))
        if not h:
            raise ValueError(f"slot {slot} is not admitted")
        cur = Tuning()
        check(self._lib.pme_get_tuning(ctypes.c_void_p(h), ctypes.byref(cur)), "pme_get_tuning")
        t = Tuning(cur.conv if conv is None else int(conv), cur.interp if interp is None else int(interp),
                   cur.bin_chunk if bin_chunk is None else int(bin_chunk))
        check(self._lib.pme_set_tuning(ctypes.c_void_p(h), ctypes.byref(t)), "pme_set_tuning")
        # the bound arguments carry the variants: rebind with the same inputs
        check(self._lib.pme_batch_update(self._h, int(slot), None, None, int(self._n[slot]),
                                         _box9(self._box[slot]), None, None), "pme_batch_update")

    def tuning_of(self, slot):
        h = self._lib.pme_batch_plan(self._h, int(slot))
        if not h:
            raise ValueError(f"slot {slot} is not admitted")
        t = Tuning()
        check(self._lib.pme_get_tuning(ctypes.c_void_p(h), ctypes.byref(t)), "pme_get_tuning")
        return t.as_dict()

    def launch_us(self, launches=5, reps=3):
        """Microseconds per pme_batch_launch of every admitted system: one
        graph of `launches` launches replayed on the pool's stream, best of
        `reps`."""
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            for _ in range(launches):
                self.launch()
        best = float("inf")
        with torch.cuda.stream(self.stream):
            g.replay()
            for _ in range(reps):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                torch.cuda._sleep(250000)  # untimed: the graph is submitted meanwhile
                a.record(self.stream)
                g.replay()
                b.record(self.stream)
                b.synchronize()
                best = min(best, a.elapsed_time(b) * 1e3 / launches)
        del g
        return best

    def autotune(self, launches=5):
        """Kernel variants per grid group chosen on the whole batch: starting
        from each plan's own variants, the groups are visited largest first
        (atoms) and each takes the (convolution, interpolation) variant under
        which the graph-replayed launch of the batch is fastest, the other
        groups held.  Returns {"us": final, "default_us": initial,
        "groups": {grid: tuning}}."""
        groups = {}
        for s in self._io:
            groups.setdefault(tuple(self._grid[s]) + (self._order[s], self._prec[s]), []).append(s)
        base = self.launch_us(launches)
        best_us = base
        order = sorted(groups, key=lambda k: -sum(self._n[s] for s in groups[k]))
        chosen = {}
        for key in order:
            slots = groups[key]
            K1, K2, K3, p, prec = key
            v = int(self._lib.pme_tuning_variants(K1, K2, K3, p, prec))
            cur = self.tuning_of(slots[0])
            best_t = dict(cur)
            for conv, cbit in ((0, 1), (1, 2), (2, 16)):
                for interp, ibit in ((0, 4), (1, 8)):
                    if not (v & cbit and v & ibit):
                        continue
                    if conv == best_t["conv"] and interp == best_t["interp"]:
                        continue
                    for s in slots:
                        self.set_tuning(s, conv=conv, interp=interp)
                    us = self.launch_us(launches)
                    if us < best_us:
                        best_us, best_t = us, {"conv": conv, "interp": interp,
                                               "bin_chunk": cur["bin_chunk"]}
            for s in slots:
                self.set_tuning(s, **best_t)
            chosen["x".join(map(str, key[:3]))] = best_t
        return {"us": best_us, "default_us": base, "groups": chosen}

    def check(self, slot):
        """Synchronise; the sticky device flags of a slot's plan (cleared)."""
        h = self._lib.pme_batch_plan(self._h, int(slot))
        if not h:
            raise ValueError(f"slot {slot} is not admitted")
        flags = ctypes.c_uint(0)
        self._lib.pme_check(ctypes.c_void_p(h), ctypes.byref(flags))
        return int(flags.value)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._lib.pme_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
