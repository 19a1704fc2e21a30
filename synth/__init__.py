"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package only draws inputs (genotypes, kinship, covariates, phenotypes and
variance components) with the shapes and distributions of the simulated GWAS
scenarios in the paper's supplementary notes (simulated data, scenario C).  It
holds none of the association method's arithmetic.
"""
from .genotypes import snp_genotypes, allele_thresholds
from .workloads import CONFIGS, Workload, make_workload, cohort_workloads
from .bedfile import pack_rows, write_bed

__all__ = ["snp_genotypes", "allele_thresholds", "CONFIGS", "Workload",
           "make_workload", "cohort_workloads", "pack_rows", "write_bed"]
