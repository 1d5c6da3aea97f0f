"""CPU oracle for checkerboard Metropolis sweeps of the 2D Ising model.

TEST INFRASTRUCTURE. Only tests/, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. It shares no
code with the HIP library in ``paper_cs_0312006_amd``.

``oracle.ref`` wraps the plain C oracle (``ising_oracle.c``);
``oracle.mini`` is a second, independently written NumPy version used to
cross-check the C one on small lattices.
"""
