"""MI355X-native implicit boundary integral method (IBIM) for the linearized
Poisson–Boltzmann equation (Zhong, Ren, Tsai, arXiv:1709.08070).

The compute path is the C-ABI HIP library ``libpb.so`` (declared in include/pb.h);
``paper_1709_08070_amd.pb`` is its thin Python binding and ``synth`` draws the seeded
synthetic molecules.
"""
