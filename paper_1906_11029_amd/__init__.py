"""MI355X-native explicit mapped tent pitching (MTP) with structure-aware Taylor time
stepping for DG Maxwell.  The compute path is the C-ABI library libmtp.so (HIP kernels
for gfx950); ``paper_1906_11029_amd.mtp`` is its thin Python binding."""
