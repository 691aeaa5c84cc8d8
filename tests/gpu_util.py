"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import sys

import pytest
import torch

DEV = "cuda:0"


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()
