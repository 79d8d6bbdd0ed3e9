"""CPU oracle of the coupled LBM-PSM-DEM step (test infrastructure only)."""
