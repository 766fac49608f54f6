"""Helpers shared by the GPU parity tests (upload, error measures)."""

import numpy as np
import torch

from paper_2102_12739_amd import workload as wl

# Parity bar for float32 arithmetic against the float64 oracle: relative L2
# error of the output vector. A 256-term float32 dot product with ~N(0,1)
# terms carries a relative rounding error of about sqrt(256) * 2^-24 ~ 1e-6
# of the term magnitudes; 1e-5 leaves room for cancellation.
REL_L2_FP32 = 1e-5


def device():
    return torch.device("cuda:0")


def rel_l2(got, ref) -> float:
    got = np.asarray(got, dtype=np.complex128)
    ref = np.asarray(ref, dtype=np.complex128)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / (den if den > 0 else 1.0))


def upload(p, grid_dtype="c64", gcf_dtype="f32"):
    dev = device()
    out = {}
    if p.subgrids is not None:
        st = wl.complex_to_storage(p.subgrids, grid_dtype)
        if grid_dtype == "c64":
            out["sub"] = torch.from_numpy(np.ascontiguousarray(p.subgrids)).to(dev)
        elif grid_dtype == "cbf16":
            out["sub"] = torch.from_numpy(st.view(np.int16)).to(dev).view(torch.bfloat16)
        else:
            out["sub"] = torch.from_numpy(st).to(dev)
    out["g_uv"] = table_tensor(p.g_uv, gcf_dtype)
    out["g_w"] = table_tensor(p.g_w, gcf_dtype)
    out["uvw"] = torch.from_numpy(np.ascontiguousarray(p.uvw)).to(dev)
    return out


def table_tensor(t, gcf_dtype):
    """A GCF table on the device in the given storage dtype."""
    st = wl.table_to_storage(t, gcf_dtype)
    if gcf_dtype == "bf16":
        return torch.from_numpy(st.view(np.int16)).to(device()).view(torch.bfloat16)
    return torch.from_numpy(st).to(device())


def stored_reference_inputs(p, grid_dtype, gcf_dtype):
    """Subgrids and tables as the library receives them, widened to float64:
    what the oracle must be given for a parity check of low-precision storage."""
    sub = p.subgrids if grid_dtype == "c64" else \
        wl.storage_to_complex128(wl.complex_to_storage(p.subgrids, grid_dtype), grid_dtype)
    g_uv, g_w = wl.stored_tables(p, gcf_dtype)
    return sub, g_uv, g_w


def plan_for(p, **kw):
    from paper_2102_12739_amd.degrid import Plan
    return Plan(p.offsets, p.n_v, p.n_u, p.n_w, p.os_uv, p.os_w, **kw)


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
