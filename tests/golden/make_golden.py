"""Writes the closed-form golden fixtures in this folder.

Uses closed forms only (no oracle, no GPU path):
* kac_n8.txt        -- Kac-Sylvester-Clement matrix, eigenvalues -(n-1), -(n-3), ..., n-1
                       (Clement 1959; Taussky & Todd 1991)
* laplacian_n12.txt -- tridiag(-1, 2, -1), eigenvalues 2 - 2 cos(k pi/(n+1))
                       (Golub & Van Loan, Section 4.8)
* torus_L4.txt      -- clean nearest-neighbour hopping t = -1 on a 4 x 4 torus,
                       eigenvalues 2t cos(2 pi kx/L) + 2t cos(2 pi ky/L)
"""
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def write(name, header, values):
    with open(os.path.join(HERE, name), "w") as f:
        for line in header:
            f.write("# " + line + "\n")
        for v in values:
            f.write(repr(float(v)) + "\n")


def main():
    n = 8
    write("kac_n8.txt",
          ["Kac-Sylvester-Clement matrix, n = 8: zero diagonal, off-diagonals sqrt(i (n - i))",
           "eigenvalues -(n-1), -(n-3), ..., n-1 (closed form; Clement 1959)"],
          [-(n - 1) + 2 * k for k in range(n)])
    n = 12
    write("laplacian_n12.txt",
          ["1-D Laplacian tridiag(-1, 2, -1), n = 12",
           "eigenvalues 2 - 2 cos(k pi/(n+1)), k = 1..n (closed form)"],
          sorted(2 - 2 * math.cos(k * math.pi / (n + 1)) for k in range(1, n + 1)))
    L = 4
    vals = sorted(-2 * math.cos(2 * math.pi * kx / L) - 2 * math.cos(2 * math.pi * ky / L)
                  for kx in range(L) for ky in range(L))
    write("torus_L4.txt",
          ["tight-binding Hamiltonian, hopping t = -1, 4 x 4 periodic lattice, zero on-site",
           "eigenvalues -2 cos(2 pi kx/L) - 2 cos(2 pi ky/L), kx, ky = 0..L-1 (closed form)"],
          vals)


if __name__ == "__main__":
    main()
