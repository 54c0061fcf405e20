"""Oracle for the staggered-grid P_N scheme (Seibold & Frank, arXiv 1211.2205).

TEST INFRASTRUCTURE.  This package is a plain, slow FP64 CPU implementation
of what the GPU library computes.  Only tests/, the smoke check in
__graft_entry__ and the CPU-baseline leg of bench.py may import it; the
product path (paper_1211_2205_amd) never imports, links or executes it, and
the two share no code.  Modules:
  pn      moment list, complex and real moment matrices, slab matrix,
          grid classes, spectral radius and time step (Sects. 2-4)
  scheme  the half-step operators and the time loop (Sects. 4-5), driving a
          plain C implementation (starmap_oracle.c) of the differences and the
          exact sub-step update
  mlp     the learned-closure network: forward, hand-written backward, Adam,
          optional bfloat16 rounding of the matrix-product operands
  closure the learned closure of P_5: input features, order-6 flux targets,
          closure terms and the closure solver
"""
