"""The entry point that allocates nothing (slice_occupancy_loss_static),
called through the C ABI, against the allocating slice_occupancy_loss on the
same inputs: two calls in a row, the second on a smaller input (the static
scratch keeps the first call's contents)."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2101_05031_amd import _native as N
from paper_2101_05031_amd import api, synth

from gpu_util import bin_lattice

pytestmark = pytest.mark.gpu


def test_static_scratch_loss_equals_the_allocating_entry_point():
    lat = synth.kuhn_lattice(3, 12.0, seed=13)
    grid = synth.grid_for(lat, 131, 117, 9, dz=0.9)
    b = bin_lattice(lat, grid)
    tau = 0.05
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    for nk in (9, 4):
        print(f"static scratch loss: nk={nk}", flush=True)
        field = api.slice_field(b, 0, nk)
        target = torch.from_numpy(np.random.default_rng(nk).uniform(
            0.0, 1.0, size=(nk, grid.H, grid.W)).astype(np.float32)).cuda()
        ref_loss, ref_grad = api.slice_occupancy_loss(b, field, target, tau)
        loss = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        grad = torch.full_like(field, -1.0)
        st = N.lib().slice_occupancy_loss_static(
            b.handle, nk, ctypes.c_void_p(field.data_ptr()), ctypes.c_void_p(target.data_ptr()),
            ctypes.c_double(tau), ctypes.c_void_p(grad.data_ptr()),
            ctypes.c_void_p(loss.data_ptr()), stream)
        assert st == N.LSL_OK, N.lib().lsl_last_error().decode()
        torch.cuda.synchronize()
        assert float(ref_loss) > 0
        # the same kernels over the same blocks: bitwise the same results
        assert torch.equal(loss, ref_loss)
        assert torch.equal(grad, ref_grad)
