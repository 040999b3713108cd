"""CPU oracle for the FFT-based psi_r / SCV hot path (test infrastructure).

THIS PACKAGE IS TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The HIP library never calls it and shares no code, table or
constant generator with it.

It is a plain, slow, float64 NumPy implementation of what the paper's method
computes (Gramacki & Gramacki, "FFT-based fast bandwidth selector for
multivariate kernel density estimation"):

* ``grid``      grid planning (Sec. 4, Eq. (15)-(16))
* ``linbin``    multivariate linear binning, bit-exact fixed-point contract
                (Sec. 4, first step; Eq. (14))
* ``gauss``     Gaussian density and its partial derivatives D^alpha phi_Sigma
                (Sec. 5, Eq. (13), (23)-(24))
* ``multiindex`` ordering of the unique entries of D^{(x)r} (Sec. 5)
* ``direct``    the unbinned double sum psi_r (Eq. (12)-(13)), O(n^2)
* ``binned``    the binned double sum (Eq. (14)) evaluated directly in the lag
                domain, with no FFT (Eq. (17)-(18) with the inner sum written
                out as an autocorrelation of the counts)
* ``layout``    the paper's literal four steps with its zero-padded layout
                (Eq. (19)-(24)), using numpy.fft as a library primitive
* ``scv``       the smoothed cross-validation objective and its gradient
                (the SCV selector is named in Sec. 3 and Sec. 5; its formula
                is the standard Gaussian-kernel SCV, read as a V-statistic)
* ``plugin``    the plug-in (AMISE) objective built on psi_4 and its gradient
                (Sec. 5 names the PI selector; standard normal-kernel AMISE)
* ``eta``       the scalar functions eta_r of Eq. (30)-(31), the V-statistic
                Q_r of Eq. (32), LSCV_r of Eq. (35)-(36) and the LSCV gradient

Pins (what ties this code to the paper and to mathematics rather than to
itself) live in ``tests/test_oracle_*.py``.
"""
from . import multiindex, grid, linbin, gauss, direct, binned, layout, scv, plugin, eta  # noqa: F401
