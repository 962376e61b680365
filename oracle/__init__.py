"""FP64 CPU oracle of the MLP-Splatting render path.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's cpu_baseline leg.  The product path (paper_2606_03877_amd) never
imports it and shares no code with it.
"""
from .render import (Model, Opts, quat_to_rotmat, local_frame, intersect, encode, mlp_apply,
                     bf16_round, split_bf16, gate_preacts, relu_noise, relu_margin, packet_centres, render, TETRA,
                     slot_gates)
from .pcg import pcg_hash, sample_offsets
from .grad import loss_and_grads, complex_step, to_tensors
from .octree import octree_leaves, octree_primitives, ssim
from .contact import (KAPPA, ContactModel, encode_vec, contact_terms, render_contact, contact_margins,
                      contact_loss_and_grads)

__all__ = ["Model", "Opts", "quat_to_rotmat", "local_frame", "intersect", "encode",
           "mlp_apply", "bf16_round", "split_bf16", "gate_preacts", "relu_noise", "relu_margin", "packet_centres", "render", "TETRA", "slot_gates", "pcg_hash", "sample_offsets", "loss_and_grads",
           "complex_step", "to_tensors", "KAPPA", "ContactModel", "encode_vec", "contact_terms",
           "render_contact", "contact_margins", "contact_loss_and_grads", "octree_leaves", "octree_primitives",
           "ssim"]
