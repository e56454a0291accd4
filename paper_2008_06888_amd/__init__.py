"""MI355X-native tropical tensor-network contraction for Ising spin glasses.

The compute path lives in the HIP library ``libtt.so`` (sources under ``csrc/``);
``binding`` marshals arguments to its C-ABI and ``autograd`` wraps it as a
``torch.autograd.Function``. ``instances`` draws seeded synthetic problems.
Submodules are imported explicitly; importing the package loads nothing native.
"""
