"""MI355X (gfx950) isothermal two-phase PT flash with the SRK equation of state.

The compute path is the HIP library built from ``csrc/`` (C ABI in
``include/ptflash.h``); this package only binds it to PyTorch tensors.
"""
from . import _capi  # noqa: F401
from .api import (FlashResult, eval_phase, flash, flash_autograd, flash_backward,  # noqa: F401
                  flash_ragged, hint_from_probability, stability)

__all__ = ["flash", "flash_ragged", "stability", "hint_from_probability", "flash_backward", "flash_autograd",
           "eval_phase", "FlashResult"]
