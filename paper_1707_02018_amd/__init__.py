"""MI355X (gfx950) implementation of the deblurring operator A = R W, its
adjoint A^* = W^* R^*, FISTA on eq. (1), and the blind-channel convolution
adjoint pair of Folberth & Becker, "Efficient Adjoint Computation for Wavelet
and Convolution Operators" (IEEE SPM Lecture Notes, 2016).

The compute path is libadjwave.so (hand-written HIP, C ABI in
include/adjwave.h); ``paper_1707_02018_amd.ops`` marshals torch device tensors
into it.
"""
