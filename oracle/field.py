"""Uniform applied field h_e(t) and its time derivative (oracle; test infrastructure only).

The paper takes the external field uniform (Sec. 2.1 for films, Sec. 3.1 for
bulk samples) and ramps it, h_e = t (Sec. 2.3 and 3.2), or drives it
sinusoidally (benchmark cube, Sec. 3.2).  Three waveforms are provided:

* ``ramp``   h_e(t) = rate * t * dir
* ``sine``   h_e(t) = amp * sin(omega t) * dir
* ``rotate`` h_e(t) = amp * (cos(omega t), sin(omega t), 0)

Only h_e and dh_e/dt enter the method: the right-hand side needs dh_e/dt
(eqs. (8), (11), (15), (18)); post-processing needs h_e (Sec. 2.1, last formula).
"""
import numpy as np

RAMP, SINE, ROTATE = 0, 1, 2


class AppliedField:
    def __init__(self, kind=RAMP, direction=(0.0, 0.0, 1.0), amp=1.0, omega=1.0, rate=1.0):
        self.kind = int(kind)
        self.dir = np.asarray(direction, dtype=np.float64)
        self.amp = float(amp)
        self.omega = float(omega)
        self.rate = float(rate)

    def h(self, t):
        """h_e(t) as a 3-vector."""
        if self.kind == RAMP:
            return self.dir * (self.rate * t)
        if self.kind == SINE:
            return self.dir * (self.amp * np.sin(self.omega * t))
        if self.kind == ROTATE:
            return self.amp * np.array([np.cos(self.omega * t), np.sin(self.omega * t), 0.0])
        raise ValueError("unknown field kind")

    def hdot(self, t):
        """dh_e/dt as a 3-vector (exact derivative of ``h``)."""
        if self.kind == RAMP:
            return self.dir * self.rate
        if self.kind == SINE:
            return self.dir * (self.amp * self.omega * np.cos(self.omega * t))
        if self.kind == ROTATE:
            w = self.omega
            return self.amp * w * np.array([-np.sin(w * t), np.cos(w * t), 0.0])
        raise ValueError("unknown field kind")
