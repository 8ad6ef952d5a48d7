"""MI355X-native D3Q27 colour-fluid lattice Boltzmann library (Saito, Abe & Koyama 2017).

``lbm`` is the binding of the HIP library (C ABI in ``include/lbm.h``); ``workloads``
holds the seeded problem descriptions shared with the test oracle.  Importing the package
loads nothing native; the library is loaded on first use.
"""
