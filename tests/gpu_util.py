"""Helpers for the GPU parity tests: device region sets with padding guards."""
import numpy as np
import torch

PAD_IN = 0xA5
PAD_OUT = 0x5A


def device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm GPU"
    return torch.device("cuda:0")


def ld_for(s, extra=0):
    return (s + 15) // 16 * 16 + 16 * extra


def to_regions(X, ld=None, offset_rows=0, extra=0):
    """Copy a (rows x s) uint8 array into a device tensor whose rows have
    stride ld (>= s, multiple of 16); bytes past s hold PAD_IN.  offset_rows
    puts the region set inside a larger allocation (a nonzero base offset)."""
    rows, s = X.shape
    ld = ld or ld_for(s, extra)
    host = np.full((rows + offset_rows, ld), PAD_IN, np.uint8)
    host[offset_rows:, :s] = X
    t = torch.from_numpy(host).to(device())
    return t[offset_rows:]


def out_regions(rows, s, ld=None, extra=0):
    ld = ld or ld_for(s, extra)
    return torch.full((rows, ld), PAD_OUT, dtype=torch.uint8, device=device())


def read(t, s):
    torch.cuda.synchronize()
    h = t.cpu().numpy()
    # nothing may be written past block_bytes
    assert np.all(h[:, s:] == PAD_OUT) or np.all(h[:, s:] == PAD_IN), "write past block end"
    return h[:, :s].copy()
