"""MI355X-native Peaceman-Rachford ADI for the 2-D acoustic system
(nodal compact and staggered mimetic fourth-order finite differences).

The compute path is the HIP library ``libadi.so`` behind the C ABI declared in
``include/adi.h``; :mod:`paper_2006_07583_amd.adi` is its thin ctypes binding.
Importing the package does not load the library.
"""
