"""FP64 CPU oracle for the QED Monte Carlo particle step (Wang, Sheng, Gibbon & Li,
"Modeling of photon and pair production due to quantum electrodynamics effects in
particle-in-cell simulation", arXiv:1608.06356).

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or execute
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP path
(``paper_1608_06356_amd``) and imports nothing from it.

It is plain NumPy in float64: the Bessel functions come from their integral
representation, the spectra are the paper's Eqs. (1), (4), (5) and (6) written out,
the tables are built by quadrature, and the Monte Carlo step runs the same
algorithm as the GPU in particle-index order.

Modules
-------
constants   physical constants in the paper's normalised units
bessel      K_nu(x) and its tail integral (integral representation)
spectra     dW/dxi for formula I (Eq. 1), formula II (Eq. 4), the classical limit
            (Eq. 5) and Breit-Wheeler pairs (Eq. 6); chi_e / chi_ph (Eqs. 2-3)
tables      total rates and inverse-CDF tables in the exact layout the GPU uses
philox      Philox4x32-10 counter-based generator and the stream convention
mc          the Monte Carlo step: push, optical depth, sampling, appends,
            compaction
mlp         the surrogate network's forward/backward pass in float64

Parity status per function is stated in each module header; a function with no
independent pin says "parity unpinned".
"""
