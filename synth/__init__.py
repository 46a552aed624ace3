"""Seeded synthetic inputs (phantoms, analytic projections, counts) and the
workload / parameter tables.  Holds none of the reconstruction arithmetic."""
