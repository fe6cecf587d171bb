"""Writes closed_forms.json: exact values of the diffusion vectors on tiny graphs.

Every number here comes from a closed form worked out by hand from the
paper's definitions (no solver is run):

* PPR  f = alpha (I - (1-alpha) A D^-1)^-1 e_s          -- Eq. (2), Table 1
* Katz x* = (I - beta A)^-1 e_s                           -- Eq. (3)
* HK   f = exp(-tau (I - A D^-1)) e_s                     -- Sec. 2, "Heat Kernel"
* LocalGD on the 2-node graph moves the whole residual across the single edge
  each iteration (Eq. (9)), so r/alpha = (1-alpha)^t at alternating ends and
  the process stops at the first t with (1-alpha)^t < eps (Definition 3.1).
* the optimal SOR relaxation omega* = 2 / (1 + sqrt(1 - (1-alpha)^2))  -- Sec. 3.2.
* psi_k = sum_{j=k}^{K} tau^(j-k) k!/j! (tail weights of the Taylor levels).
"""
import json
import math
import os

out = {}
a = 0.1
out["ppr_two_node"] = dict(
    citation="Eq. (2), Table 1; graph 0-1", alpha=a, seed=0, f=[1 / (2 - a), (1 - a) / (2 - a)])
ka = a * (1 + 3 * a) / ((1 + 3 * a) - (1 - a) ** 2)
out["ppr_k5"] = dict(citation="Eq. (2); complete graph K5, seed 0", alpha=a, seed=0,
                     f=[ka] + [(1 - a) * ka / (1 + 3 * a)] * 4)
fc = 1 / (2 - a)
out["ppr_star_centre"] = dict(citation="Eq. (2); star, centre 0, leaves 1-4", alpha=a, seed=0,
                              f=[fc] + [(1 - a) * fc / 4] * 4)
fc = (1 - a) / (2 - a)
fj = (1 - a) * fc / 4
out["ppr_star_leaf"] = dict(citation="Eq. (2); star, centre 0, leaves 1-4, seed leaf 1", alpha=a, seed=1,
                            f=[fc, a + fj, fj, fj, fj])
b = 0.25
out["katz_two_node"] = dict(citation="Eq. (3); graph 0-1", beta=b, seed=0, x=[1 / (1 - b * b), b / (1 - b * b)])
tau = 5.0
out["hk_two_node"] = dict(citation="Sec. 2 Heat Kernel; graph 0-1", tau=tau, seed=0,
                          f=[math.exp(-tau) * math.cosh(tau), math.exp(-tau) * math.sinh(tau)])
K = 30
psi = []
for k in range(K + 1):
    psi.append(sum(tau ** (j - k) * math.factorial(k) / math.factorial(j) for j in range(k, K + 1)))
out["hk_psi"] = dict(citation="Sec. 2 Heat Kernel, Taylor truncation at K", tau=tau, K=K, psi=psi)
eps = 1e-6
T = next(t for t in range(10000) if (1 - a) ** t < eps)
x0 = a * sum((1 - a) ** t for t in range(0, T, 2))
x1 = a * sum((1 - a) ** t for t in range(1, T, 2))
out["localgd_two_node"] = dict(citation="Eq. (9), Definition 3.1; graph 0-1, PPR", alpha=a, eps=eps, seed=0, T=T,
                               ops=T, x=[x0, x1], residual_node=T % 2, residual=(1 - a) ** T)
out["omega_star"] = dict(citation="Sec. 3.2, optimal omega for Stieltjes Q",
                         values={str(al): 2 / (1 + math.sqrt(1 - (1 - al) ** 2)) for al in (0.1, 0.25)})
path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "closed_forms.json")
with open(path, "w") as fh:
    json.dump(out, fh, indent=1)
print(path)
