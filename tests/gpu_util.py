"""Helpers for the GPU tests: device selection and flushing progress lines."""
import sys

import pytest


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1811_03557_amd import _lib
    _lib.load()  # raises when the HIP library is missing: never a silent fallback
    return torch.device("cuda:0")


def say(msg: str) -> None:
    sys.stdout.write(msg + "\n")
    sys.stdout.flush()
