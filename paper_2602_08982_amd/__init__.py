"""MI355X (gfx950) implementation of the data-parallel TDSLDA step of the
W-SLDA Toolkit paper (arXiv 2602.08982): the C-ABI library libtdslda.so
(HIP kernels, built by paper_2602_08982_amd.build) and its ctypes binding
paper_2602_08982_amd.tdslda."""
