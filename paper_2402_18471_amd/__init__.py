"""MI355X coagulation-fragmentation hot path."""
