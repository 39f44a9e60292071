"""Host ablations of the paper's whole-operator structures (CPU, FP64, numpy).

``compressed``: the DAX and DAS compressed operators of Sec. III-A1 with their
MTP (composition by Kronecker product) and MVM (Sec. III-A2), and the dense
Matrix operator they are compared with in Figs. 6-7. They reproduce the
paper's own CPU experiments. The GPU path never builds a whole-operator
structure: it applies each gate from its gate-local form. The checker
(``oracle/``) neither uses nor is used by this package.
"""
