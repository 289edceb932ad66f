"""Convenience owner of one lattice handle and its torch-allocated state buffer."""
from __future__ import annotations

import numpy as np
import torch

from . import misa as M


class Lattice:
    """One periodic BCC box driven by libmisa on the current CUDA (HIP) device.

    The state buffer is a torch uint8 tensor owned by this object; the HIP
    stream is torch's current stream at construction.
    """

    def __init__(self, n_cells, a, rc, delta, mass, precision="fp64", runaway_capacity=0, device="cuda"):
        if isinstance(n_cells, int):
            n_cells = (n_cells,) * 3
        self.n_cells = tuple(int(k) for k in n_cells)
        self.a, self.rc, self.delta, self.mass = float(a), float(rc), float(delta), float(mass)
        self.precision = precision
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        prec = {"fp64": M.MISA_FP64, "fp32": M.MISA_FP32, "mlp": M.MISA_MLP}[precision]
        self.h = M.misa_create_lattice(self.n_cells, a, rc, delta, mass, prec, runaway_capacity,
                                       self.stream.cuda_stream)
        nbytes = M.misa_state_bytes(self.h)
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._buf.data_ptr()
        self._ptr = (base + 255) // 256 * 256
        M.misa_bind_state(self.h, self._ptr, nbytes)
        self.state_bytes = nbytes

    @property
    def box(self):
        return tuple(k * self.a for k in self.n_cells)

    def set_tables(self, tables):
        M.misa_set_potential_tables(self.h, tables["f"], tables["phi"], tables["F"])

    @classmethod
    def _adopt(cls, h, n_cells, a, rc, delta, mass, device):
        """Wrap a handle owned elsewhere (a batch box) and bind a state buffer to it."""
        self = cls.__new__(cls)
        self.n_cells = tuple(int(k) for k in n_cells)
        self.a, self.rc, self.delta, self.mass = float(a), float(rc), float(delta), float(mass)
        self.precision = "fp32"
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = h
        self._owned = False
        nbytes = M.misa_state_bytes(h)
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        self._ptr = (self._buf.data_ptr() + 255) // 256 * 256
        M.misa_bind_state(h, self._ptr, nbytes)
        self.state_bytes = nbytes
        return self

    def set_mlp(self, nets):
        """nets: {MISA_FN_F: net, MISA_FN_PHI: net, MISA_FN_EMB: net} (learned form only)."""
        for fn, net in nets.items():
            M.misa_set_mlp(self.h, fn, net)

    def set_state(self, x, v):
        M.misa_set_state(self.h, x, v)

    def get_state(self):
        return M.misa_get_state(self.h)

    def compute(self, energies=True):
        M.misa_compute_rho(self.h)
        e = torch.zeros(2, dtype=torch.float64, device=self.device) if energies else None
        M.misa_compute_force(self.h, e)
        return e

    def field(self, which):
        return M.misa_get_atom_field(self.h, which)

    def rho(self):
        return self.field(M.MISA_FIELD_RHO)

    def fprime(self):
        return self.field(M.MISA_FIELD_FPRIME)

    def forces(self):
        return self.field(M.MISA_FIELD_FORCE)

    def slots(self):
        return M.misa_debug_export(self.h, M.MISA_EXPORT_SLOTS)

    def stencil(self):
        return M.misa_debug_export(self.h, M.MISA_EXPORT_STENCIL)

    def save_checkpoint(self):
        """The whole state (bit-exact resume with load_checkpoint) as a uint8 numpy array."""
        return M.misa_save_checkpoint(self.h)

    def load_checkpoint(self, buf):
        M.misa_load_checkpoint(self.h, buf)

    def neighbour_counts(self):
        """Per atom: partners within rc as the density pass of this form counts them."""
        return M.misa_debug_export(self.h, M.MISA_EXPORT_NEIGHBOURS)

    def defects(self):
        return M.misa_defects(self.h)

    def set_pair_schedule(self, schedule):
        """"gather" (default: each pair evaluated from both ends) or "half" (Newton's
        third law: each pair once, coloured tiles; FP32 table form, axes multiple of 16)."""
        codes = {"gather": M.MISA_PAIRS_GATHER, "half": M.MISA_PAIRS_HALF}
        if schedule not in codes:
            raise ValueError(f"unknown pair schedule {schedule!r}")
        M.misa_set_pair_schedule(self.h, codes[schedule])

    def step(self, nsteps, dt_max, dx_max=0.0):
        return M.misa_step(self.h, nsteps, dt_max, dx_max)

    def set_graph(self, enable=True):
        """Steps replay a captured HIP graph (launch overhead of small boxes)."""
        M.misa_set_graph(self.h, enable)

    def set_timing(self, enable=True):
        M.misa_set_timing(self.h, enable)

    def timing(self):
        return M.misa_get_timing(self.h)

    def close(self):
        if self.h is not None and getattr(self, "_owned", True):
            M.misa_destroy_lattice(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent periodic boxes (batched replicas) stepped by misa_batch_step.

    boxes[k] is a Lattice view of box k (its handle belongs to the batch) with its
    own torch state buffer; load atoms and read results through it."""

    def __init__(self, box_cells, a, rc, delta, mass, runaway_capacity=0, device="cuda"):
        self.device = torch.device(device)
        self.stream = torch.cuda.current_stream(self.device)
        cells = [(k, k, k) if isinstance(k, int) else tuple(k) for k in box_cells]
        self.b = M.misa_batch_create(cells, a, rc, delta, mass, runaway_capacity, self.stream.cuda_stream)
        self.boxes = [Lattice._adopt(M.misa_batch_box(self.b, k), c, a, rc, delta, mass, device)
                      for k, c in enumerate(cells)]

    def __len__(self):
        return len(self.boxes)

    def set_tables(self, tables):
        M.misa_batch_set_potential_tables(self.b, tables["f"], tables["phi"], tables["F"])

    def step(self, nsteps, dt_max, dx_max=0.0, want_stats=True):
        return M.misa_batch_step(self.b, len(self.boxes), nsteps, dt_max, dx_max, want_stats)

    def set_graph(self, enable=True):
        """Batched steps replay a captured HIP graph."""
        M.misa_batch_set_graph(self.b, enable)

    def set_tile_shape(self, k, shape):
        """Tile shape of box k in the batched passes: an index into M.MISA_TILE_SHAPES."""
        M.misa_batch_set_tile_shape(self.b, k, shape)

    def tile_shape(self, k):
        return M.misa_batch_get_tile_shape(self.b, k)

    def autotune(self, probe_steps, dt_max, dx_max=0.0):
        """Choose the tile policy by timing (advances every box by the returned steps_done)."""
        return M.misa_batch_autotune(self.b, probe_steps, dt_max, dx_max)

    def close(self):
        if self.b is not None:
            for box in self.boxes:
                box.h = None
            M.misa_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
