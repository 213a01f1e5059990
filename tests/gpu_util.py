"""Upload/download and comparison helpers of the GPU parity tests.

Inputs are generated on the host (``synthetic``), rounded to the storage
precision on the host, uploaded, and the oracle is fed the same rounded values
promoted to complex128.  Nothing the GPU computes is ever an oracle input.
"""
import sys

import numpy as np
import torch

from tests.helpers import bf16_bits, f16_pairs, from_bf16_bits, from_f16_pairs

DEV = "cuda:0"

# unit roundoff of the storage formats (round to nearest even)
UNIT = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}
TOL = {"c64": 1e-5, "c128": 1e-12}


def set_knob(monkeypatch, name: str, value):
    """Set (value None: unset) a DSLASH_* tuning variable for the rest of the
    test and have the library read it again (it reads them once per process
    otherwise).  monkeypatch restores the variable when the test ends, and the
    tests' conftest has the library read it once more after that."""
    from paper_1808_05506_amd import dslash as D
    if value is None:
        monkeypatch.delenv(name, raising=False)
    else:
        monkeypatch.setenv(name, value)
    D.reload_tuning()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rounded(a: np.ndarray, dt: str) -> np.ndarray:
    """What a device buffer of storage dtype dt holds, as complex128."""
    if dt == "c64":
        return a.astype(np.complex64).astype(np.complex128)
    if dt == "c128":
        return a.astype(np.complex128)
    if dt == "bf16":
        return from_bf16_bits(bf16_bits(a))
    if dt == "f16":
        return from_f16_pairs(f16_pairs(a))
    raise ValueError(dt)


def up(a: np.ndarray, dt: str) -> torch.Tensor:
    if dt == "c64":
        return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex64))).to(DEV)
    if dt == "c128":
        return torch.from_numpy(np.ascontiguousarray(a.astype(np.complex128))).to(DEV)
    if dt == "bf16":
        return torch.from_numpy(np.ascontiguousarray(bf16_bits(a).view(np.int16))).to(DEV).view(torch.bfloat16)
    if dt == "f16":
        return torch.from_numpy(np.ascontiguousarray(f16_pairs(a))).to(DEV)
    raise ValueError(dt)


def down(t: torch.Tensor) -> np.ndarray:
    if t.dtype in (torch.complex64, torch.complex128):
        return t.cpu().numpy().astype(np.complex128)
    if t.dtype == torch.bfloat16:
        return from_bf16_bits(t.view(torch.int16).cpu().numpy().view(np.uint16))
    if t.dtype == torch.float16:
        return from_f16_pairs(t.cpu().numpy())
    raise ValueError(t.dtype)


def compare(gpu: np.ndarray, ref: np.ndarray, dt: str, label: str):
    """Element-by-element parity.

    c64 / c128: relative L2 over the whole output <= 1e-5 / 1e-12, and every
    element within tol * (|ref| + rms(ref)).
    bf16 / f16 (FP32 arithmetic, output rounded to nearest even): every element
    within u |ref| + 1e-5 rms(ref), u the unit roundoff of the format; the
    relative L2 error is reported.
    """
    diff = np.abs(gpu - ref)
    rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
    rel = float(np.linalg.norm((gpu - ref).ravel()) / np.linalg.norm(ref.ravel()))
    say(f"{label}: rel-L2 {rel:.3e}  max|diff| {diff.max():.3e}  rms(ref) {rms:.3e}")
    if dt in TOL:
        tol = TOL[dt]
        assert rel <= tol, f"{label}: rel-L2 {rel} > {tol}"
        bad = diff > tol * (np.abs(ref) + rms)
        assert not bad.any(), f"{label}: {bad.sum()} elements out of tolerance"
    else:
        bound = UNIT[dt] * np.abs(ref) + 1e-5 * rms
        bad = diff > bound
        assert not bad.any(), f"{label}: {bad.sum()} elements beyond the {dt} rounding bound"
    return rel
