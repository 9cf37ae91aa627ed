"""MI355X-native fast Walsh-Hadamard-to-boundary-wavelet operator (Antun, arXiv 2106.00554).

The compute path is the HIP library libwh2wav.so (C ABI in include/wh2wav.h);
this package only marshals arguments to it.  See `operator.Wh2Wav` for the
torch-facing wrapper and `autograd` for the differentiable form.
"""
