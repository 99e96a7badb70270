"""pyrosw: Swendsen-Wang cluster Monte Carlo on the pyrochlore lattice for MI355X."""
