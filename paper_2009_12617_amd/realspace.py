"""Real-space Ewald term on the GPU (C ABI pme_real): the erfc pair sum
within a cutoff, the self term and the exclusion correction.  Argument
marshalling only; the work runs in libspme.so."""
import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check
from .plan import _dev_f64


class RealSpace:
    """Holds the device workspace for up to max_atoms atoms and max_cells
    cells of the neighbour grid."""

    def __init__(self, max_atoms, max_cells=1 << 15, device=None):
        self._lib = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        self.max_atoms, self.max_cells = int(max_atoms), int(max_cells)
        nbytes = self._lib.pme_real_workspace_bytes(self.max_atoms, self.max_cells)
        if nbytes == 0:
            raise ValueError("bad max_atoms / max_cells")
        raw = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-raw.data_ptr()) % 256
        self._raw = raw
        self._ws = raw[off:off + nbytes]
        self._nbytes = nbytes
        self._excl_ok = None  # exclusion tensors last checked

    def __call__(self, pos, q, box, beta, rcut, exclusions=None, coulomb=1.0, forces=None,
                 accumulate=False, stream=None):
        """pos [N,3], q [N] float64 device tensors; box 3x3 host (diagonal);
        exclusions: (offsets [N+1], partners) int32 device tensors or None.
        Returns (forces [N,3], energies [3] = E_real, E_self, E_excl)."""
        n = int(q.shape[0])
        if n > self.max_atoms:
            raise ValueError(f"{n} atoms exceed this workspace's max_atoms={self.max_atoms}")
        _dev_f64(pos, (n, 3), "pos")
        _dev_f64(q, (n,), "q")
        if forces is None:
            forces = torch.empty((n, 3), dtype=torch.float64, device=self.device)
        _dev_f64(forces, (n, 3), "forces")
        energies = torch.empty(3, dtype=torch.float64, device=self.device)
        b = np.ascontiguousarray(np.asarray(box, dtype=np.float64).reshape(9))
        bp = b.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        off = idx = None
        if exclusions is not None:
            off, idx = exclusions
            for t, name in ((off, "exclusion offsets"), (idx, "exclusion partners")):
                if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.int32 \
                        or t.dim() != 1 or not t.is_contiguous():
                    raise TypeError(f"{name} must be a contiguous 1-D int32 GPU tensor")
            if off.shape[0] != n + 1:
                raise ValueError("exclusion offsets must have length N+1")
            # the partner list must hold exactly the entries the offsets index
            # (the kernels read off[0..N]); checked with one host read per
            # pair of tensors and contents, then remembered
            key = (off.data_ptr(), idx.data_ptr(), idx.numel(), off._version, idx._version)
            if key != self._excl_ok:
                ends = off[[0, -1]].cpu()
                if int(ends[0]) != 0 or int(ends[1]) != idx.numel():
                    raise ValueError("exclusion offsets must start at 0 and end at len(partners)")
                self._excl_ok = key
        s = stream if stream is not None else torch.cuda.current_stream(self.device)
        check(self._lib.pme_real(pos.data_ptr(), q.data_ptr(), n, bp, float(beta), float(rcut),
                                 float(coulomb), off.data_ptr() if off is not None else None,
                                 idx.data_ptr() if idx is not None else None, forces.data_ptr(),
                                 int(bool(accumulate)), energies.data_ptr(), self._ws.data_ptr(),
                                 self._nbytes, self.max_atoms, self.max_cells, s.cuda_stream),
              "pme_real")
        return forces, energies
