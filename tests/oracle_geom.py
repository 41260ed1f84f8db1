"""Maps the shared workload geometries onto the oracle's geometry classes."""
from oracle import geometry


def oracle_geometry(g):
    if g.kind == "balls":
        return geometry.Balls(g.centers, g.radii)
    return geometry.Star2D(g.star_r0, g.star_a, g.star_k)
