"""MI355X-native hot path of the Gaia astrometric core solution (AGIS).

The HIP library ``libagis.so`` (built from ``csrc/`` by ``build.py``)
implements the source, attitude and calibration updating blocks and the
frame rotator; ``agis`` is its ctypes binding.
"""
