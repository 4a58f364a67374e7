"""Writes the closed-form fixtures in this folder (pure ``math``; no model code).

one_pixel.json: a 1x1 frame, one mode, one slice, one position. The unitary 1x1 DFT
is the identity, so Psi = p * o and I = |p o|^2, and the losses and their gradients
(g = dL/dRe + i dL/dIm) have closed forms:
  amplitude (Eq. (1) with B = H = W = 1): L = (|p o| - sqrt(Im))^2,
      g_o = 2 (1 - sqrt(Im / I)) conj(p) p o,  g_p = 2 (1 - sqrt(Im / I)) conj(o) o p
  Poisson:  L = I - Im ln(I + eps),
      g_o = 2 (1 - Im / (I + eps)) conj(p) p o, g_p likewise with o and p swapped.
plane_wave.json: object exp(2 pi i (u y + v x) / N), probe of ones, position (0, 0):
  the far field is one bright bin of value N^2 at the centred index
  ((u + N/2) mod N, (v + N/2) mod N); every other bin is 0.
"""
import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def one_pixel():
    cases = []
    # amplitude loss
    p, o, im = complex(1, 1), complex(0.5, 0), 2.0
    I = abs(p * o) ** 2
    c = 1.0 - math.sqrt(im / I)
    L = (math.sqrt(I) - math.sqrt(im)) ** 2
    go = 2 * c * p.conjugate() * p * o
    gp = 2 * c * o.conjugate() * o * p
    cases.append(dict(loss="amplitude", eps=0.0, p=[p.real, p.imag], o=[o.real, o.imag], I_meas=im,
                      L=L, I=I, g_obj=[go.real, go.imag], g_probe=[gp.real, gp.imag]))
    # Poisson loss
    p, o, im, eps = complex(2, 0), complex(1, -1), 5.0, 1e-3
    I = abs(p * o) ** 2
    c = 1.0 - im / (I + eps)
    L = I - im * math.log(I + eps)
    go = 2 * c * p.conjugate() * p * o
    gp = 2 * c * o.conjugate() * o * p
    cases.append(dict(loss="poisson", eps=eps, p=[p.real, p.imag], o=[o.real, o.imag], I_meas=im,
                      L=L, I=I, g_obj=[go.real, go.imag], g_probe=[gp.real, gp.imag]))
    return dict(source="closed forms of Eq. (1) and the Poisson reading on a 1x1 frame; Sec. 2.2",
                cases=cases)


def plane_wave():
    out = []
    for (N, u, v) in [(8, 1, 3), (16, 5, 0), (16, 15, 9)]:
        out.append(dict(N=N, u=u, v=v, bright=[(u + N // 2) % N, (v + N // 2) % N], value=float(N * N)))
    return dict(source="far-field of a plane wave under the unitary DFT with DC-centred detector", cases=out)


if __name__ == "__main__":
    with open(os.path.join(HERE, "one_pixel.json"), "w") as f:
        json.dump(one_pixel(), f, indent=1)
    with open(os.path.join(HERE, "plane_wave.json"), "w") as f:
        json.dump(plane_wave(), f, indent=1)
